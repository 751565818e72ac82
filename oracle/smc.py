"""SMC-sampler and population-MCMC steps, plain FP64 definitions.

Sections of the paper followed here:
  * Sequential Monte Carlo / SMC Samplers: weighted particles, resampling by
    building the empirical CDF of the normalised weights and drawing N times
    from it, triggered by an effective-sample-size criterion.
  * SMC Sampler (Mixture Modelling): tempered targets pi_t ~ pi^{beta_t}, an
    initial population from the prior, random-walk Metropolis-Hastings moves
    at every step, and (with a pi_t-invariant move and the generic backward
    kernel) incremental weights pi_t(x_{t-1}) / pi_{t-1}(x_{t-1}).
  * Population-Based MCMC: M chains targeting pi^{beta_i}, stage-one moves in
    parallel, then exchange moves between adjacent chains on disjoint pairs,
    accepted with probability min(1, alpha_ij) where
    alpha_ij = pi_i(x_j) pi_j(x_i) / (pi_i(x_i) pi_j(x_j)).
  * Importance Sampling: normalised weights W = w / sum w.

Readings where the paper is silent or ambiguous (each one is listed in the
design notes):
  * Tempering acts on the likelihood only: pi_beta ~ p0 * L^beta. With the
    paper's uniform prior this equals pi^beta on the box; with a Gaussian prior
    it is the only reading under which beta = 0 is the prior the sampler starts
    from. The incremental weight is then L(x)^{dbeta}.
  * Step order: reweight, then resample if ESS < ess_frac * N (strict), then
    the RW-MH moves at the new temperature; the same rule applies at t = T.
  * Resampling scheme: systematic (the paper does not name one).
  * log-evidence: log Z = sum_t log sum_p W_p^{(t-1)} exp(dbeta_t * l_p), the
    standard SMC-sampler estimator (not computed in the paper).
"""

from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from . import philox as px
from .gmm import Model, log_prior, loglik


# ---------------------------------------------------------------------------
# weights

def lse(v) -> float:
    """log sum exp(v) with max shift; -inf for an empty or all -inf vector."""
    v = np.asarray(v, dtype=np.float64)
    if v.size == 0:
        return -math.inf
    m = float(np.max(v))
    if m == -math.inf:
        return -math.inf
    return m + math.log(float(np.sum(np.exp(v - m))))


def normalise(logw):
    """Normalised weights W_p = exp(logw_p - m) / sum_q exp(logw_q - m)."""
    logw = np.asarray(logw, dtype=np.float64)
    if not np.all(np.isfinite(logw) | (logw == -np.inf)) or np.all(logw == -np.inf):
        raise FloatingPointError("log-weights are NaN, +inf or all -inf")
    m = np.max(logw)
    e = np.exp(logw - m)
    return e / np.sum(e)


def ess(W) -> float:
    """Effective sample size 1 / sum W^2 of normalised weights."""
    W = np.asarray(W, dtype=np.float64)
    return 1.0 / float(np.sum(W * W))


def reweight(logw, l, dbeta):
    """Incremental reweight for a tempering step.

    logw_new = logw + dbeta * l (the log of L(x)^dbeta), normalised weights W,
    the log-evidence increment log sum_p W_p^{old} exp(dbeta l_p), which equals
    lse(logw_new) - lse(logw_old), and ESS.
    Returns (logw_new, W, logZ_increment, ess).
    """
    logw = np.asarray(logw, dtype=np.float64)
    l = np.asarray(l, dtype=np.float64)
    lse_old = lse(logw)
    logw_new = logw + dbeta * l
    W = normalise(logw_new)
    lse_new = lse(logw_new)
    return logw_new, W, lse_new - lse_old, ess(W)


# ---------------------------------------------------------------------------
# systematic resampling

def prefix_sums_correctly_rounded(W) -> np.ndarray:
    """C_j = the double nearest to the exact sum W_0 + ... + W_j.

    The partial sums are accumulated exactly as integers (every double is an
    integer multiple of 2^-1074) and each one is rounded once, by CPython's
    correctly rounded integer true division.
    """
    W = np.asarray(W, dtype=np.float64)
    if np.any(W < 0) or not np.all(np.isfinite(W)):
        raise ValueError("weights must be finite and non-negative")
    mant, ex = np.frexp(W)
    M = (mant * 2.0 ** 53).astype(np.int64)          # exact: |mant| < 1
    e = ex.astype(np.int64) - 53
    base = int(e.min()) if W.size else 0
    shift = (e - base).tolist()
    Ml = M.tolist()
    den = 1 << (-base) if base < 0 else 1
    num_scale = 1 << base if base > 0 else 1
    out = np.empty(W.size, dtype=np.float64)
    acc = 0
    for j in range(W.size):
        acc += Ml[j] << shift[j]
        out[j] = (acc * num_scale) / den
    return out


def systematic_offsets(N, u) -> np.ndarray:
    """U_i = (i + u) / N in FP64 (i + u is exact for N <= 2^21; one rounding)."""
    i = np.arange(N, dtype=np.float64)
    return (i + u) / float(N)


def systematic_resample(W, u) -> np.ndarray:
    """Ancestor indices idx_i = min{j : U_i < C_j}.

    C is the correctly rounded empirical CDF of W, U_i = (i + u)/N with
    u in [0, 1). If rounding leaves U_i >= C_{N-1}, idx_i is the first j with
    C_j = C_{N-1} (the last particle of positive weight). Zero-weight
    particles are never selected. Returns int32 indices, non-decreasing.
    """
    W = np.asarray(W, dtype=np.float64)
    N = W.size
    C = prefix_sums_correctly_rounded(W)
    U = systematic_offsets(N, u)
    idx = np.searchsorted(C, U, side="right")        # first j with U < C_j
    last = int(np.searchsorted(C, C[-1], side="left"))
    idx = np.where(idx >= N, last, idx)
    return idx.astype(np.int32)


# Resampling schemes (Sequential Monte Carlo subsection: the new population is
# drawn from the empirical CDF of the weights). All three take
# idx_i = min{j : U_i < C_j} on the same correctly rounded CDF, with the same
# clamp, and differ only in the points U_i:
#   systematic   U_i = (i + u) / N, one u per step;
#   stratified   U_i = (i + u_i) / N, one u_i per stratum i;
#   multinomial  U_i = u_i, N independent uniforms ("sampling N times").
SCHEMES = ("systematic", "stratified", "multinomial")


def per_index_uniforms(seed, step, N, scheme):
    """u_i in [0, 1) for stratified (scheme code 1) or multinomial (code 2)
    resampling: 53-bit uniforms from words 0, 1 of stream (i, 0, step, RESAMP, code)."""
    code = SCHEMES.index(scheme)
    w0, w1, _, _ = px.words(seed, np.arange(N, dtype=np.uint64), 0, step, px.RESAMP, code)
    return px.u01_53(w0, w1)


def resample_points(N, scheme, seed, step):
    """The points U_i of a scheme in FP64 (each a single rounding of its formula)."""
    if scheme == "systematic":
        return systematic_offsets(N, resample_offset(seed, step))
    u = per_index_uniforms(seed, step, N, scheme)
    if scheme == "stratified":
        return (np.arange(N, dtype=np.float64) + u) / float(N)
    if scheme == "multinomial":
        return u
    raise ValueError(f"unknown resampling scheme {scheme!r}")


def search_cdf(W, U) -> np.ndarray:
    """idx_i = min{j : U_i < C_j} on the correctly rounded CDF of W; U_i >= C_{N-1}
    (possible only through rounding) maps to the first j with C_j = C_{N-1}."""
    W = np.asarray(W, dtype=np.float64)
    C = prefix_sums_correctly_rounded(W)
    idx = np.searchsorted(C, U, side="right")
    last = int(np.searchsorted(C, C[-1], side="left"))
    return np.where(idx >= W.size, last, idx).astype(np.int32)


def resample_indices(W, scheme, seed, step) -> np.ndarray:
    """Ancestor indices of one resampling under `scheme`."""
    W = np.asarray(W, dtype=np.float64)
    return search_cdf(W, resample_points(W.size, scheme, seed, step))


def search_bruteforce(W, U):
    """Exact-rational search for tiny N: C_j and the given U_i as fractions,
    linear scan, the same clamp."""
    Wf = [Fraction(float(w)) for w in W]
    C, acc = [], Fraction(0)
    for w in Wf:
        acc += w
        C.append(acc)
    out = []
    for Ui in U:
        Uf = Fraction(float(Ui))
        j = next((j for j in range(len(W)) if Uf < C[j]), None)
        if j is None:
            j = next(j for j in range(len(W)) if C[j] == C[-1])
        out.append(j)
    return np.asarray(out, dtype=np.int32)


def systematic_resample_bruteforce(W, u):
    """Exact-rational version for tiny N: the same definition with U_i, C_j as
    exact fractions and a linear scan."""
    N = len(W)
    Wf = [Fraction(float(w)) for w in W]
    C = []
    acc = Fraction(0)
    for w in Wf:
        acc += w
        C.append(acc)
    uf = Fraction(float(u))
    out = []
    for i in range(N):
        Ui = (i + uf) / N
        j = next((j for j in range(N) if Ui < C[j]), None)
        if j is None:
            j = next(j for j in range(N) if C[j] == C[-1])
        out.append(j)
    return np.asarray(out, dtype=np.int32)


def resample_offset(seed, step) -> float:
    """The per-step systematic-resampling offset u in [0, 1)."""
    w0, _, _, _ = px.words(seed, 0, 0, step, px.RESAMP, 0)
    return float(px.u01_left_closed(w0))


# ---------------------------------------------------------------------------
# prior draws and the random-walk Metropolis-Hastings move

def prior_init(model: Model, N: int, seed: int) -> np.ndarray:
    """theta_0 from the prior, layout [k*d][N]."""
    kd = model.k * model.d
    idx = np.arange(N, dtype=np.uint64)
    if model.prior == "gauss":
        z = px.normals(seed, idx, 0, px.PRIOR, 0, kd)
        return model.prior_a + model.prior_b * z
    if model.prior == "box":
        nb = (kd + 3) // 4
        out = np.empty((4 * nb, N))
        for b in range(nb):
            ws = px.words(seed, idx, b, 0, px.PRIOR, 0)
            for q in range(4):
                out[4 * b + q] = model.prior_a + (model.prior_b - model.prior_a) * px.u01_open(ws[q])
        return out[:kd]
    raise ValueError(model.prior)


def rwmh_log_alpha(beta, l_cur, l_prop, lp_cur, lp_prop):
    """log of the MH ratio for the tempered target p0 * L^beta with a symmetric
    random-walk proposal."""
    return beta * (l_prop - l_cur) + (lp_prop - lp_cur)


def rwmh_move(theta, l, y, model: Model, beta, step_sd, seed, step, move, index=None):
    """One random-walk MH move of every particle, N(0, I) scaled by step_sd,
    jointly over all k*d coordinates. ``beta`` is a scalar or one value per
    particle (per chain, for parallel tempering). Column p is particle
    ``index[p]`` of the population (default: p), whose number selects its
    random streams. Returns (theta, l, accepted)."""
    theta = np.array(theta, dtype=np.float64, copy=True)
    l = np.array(l, dtype=np.float64, copy=True)
    kd, N = theta.shape
    idx = (np.arange(N, dtype=np.uint64) if index is None
           else np.asarray(index, dtype=np.uint64))
    z = px.normals(seed, idx, step, px.PROP, move, kd)
    prop = theta + step_sd * z
    l_prop = loglik(prop, y, model)
    la = rwmh_log_alpha(np.asarray(beta, dtype=np.float64), l, l_prop,
                        log_prior(theta, model), log_prior(prop, model))
    u = px.uniforms_open(seed, idx, step, px.ACC, move)
    accept = (la >= 0.0) | (np.log(u) < la)
    theta[:, accept] = prop[:, accept]
    l[accept] = l_prop[accept]
    return theta, l, accept


# ---------------------------------------------------------------------------
# SMC sampler

def _reweight_resample(theta, l, logw, betas, t, seed, ess_frac, resample, scheme):
    """The first part of tempering step t: reweight by L^(beta_t - beta_{t-1});
    if ESS < ess_frac * N resample (points from the streams of step t) and reset
    the log-weights. Returns (theta, l, logw, W, logZ_increment, info, idx)
    with idx the ancestor of each position (None without resampling)."""
    N = l.size
    dbeta = betas[t] - betas[t - 1]
    logw, W, inc, e = reweight(logw, l, dbeta)
    did = bool(resample and e < ess_frac * N)
    u = None
    idx = None
    if did:
        u = resample_offset(seed, t) if scheme == "systematic" else None
        idx = resample_indices(W, scheme, seed, t)
        theta = theta[:, idx]
        l = l[idx]
        logw = np.zeros(N)
        W = np.full(N, 1.0 / N)
    return theta, l, logw, W, inc, dict(ess=e, resampled=did, u=u), idx


def smc_step(theta, l, logw, y, model: Model, betas, t, step_sd, n_moves, seed,
             ess_frac=0.5, resample=True, scheme="systematic"):
    """Tempering step t >= 1: reweight by L^(beta_t - beta_{t-1}); if
    ESS < ess_frac * N resample (systematic by default; points from the streams
    of step t) and reset the log-weights; then n_moves RW-MH moves at beta_t
    (move m uses stream move m). Returns (theta, l, logw, W, logZ_increment, info)."""
    theta, l, logw, W, inc, info, _ = _reweight_resample(theta, l, logw, betas, t, seed,
                                                         ess_frac, resample, scheme)
    accepted = []
    for m in range(n_moves):
        theta, l, a = rwmh_move(theta, l, y, model, betas[t], step_sd, seed, t, m)
        accepted.append(a)
    info["accepted"] = accepted
    return theta, l, logw, W, inc, info


def smc_step_sampled(theta, l, logw, y, model: Model, betas, t, step_sd, n_moves, seed,
                     sample, ess_frac=0.5, resample=True, scheme="systematic"):
    """smc_step with the moves taken only by the particles at positions
    ``sample`` of the (resampled) population. A particle's moves depend on its
    own state and its own streams only, so these are exactly the corresponding
    columns of smc_step's result; the reweight, evidence, ESS and resampling
    are over the whole population as there. Returns (theta_s [kd][len(sample)],
    l_s, logw, W, logZ_increment, info); info["ancestor"] holds the ancestor of
    each sampled position (the position itself without resampling)."""
    sample = np.asarray(sample, dtype=np.int64)
    theta, l, logw, W, inc, info, idx = _reweight_resample(theta, l, logw, betas, t, seed,
                                                           ess_frac, resample, scheme)
    th_s, l_s = theta[:, sample], l[sample]
    accepted = []
    for m in range(n_moves):
        th_s, l_s, a = rwmh_move(th_s, l_s, y, model, betas[t], step_sd, seed, t, m,
                                 index=sample)
        accepted.append(a)
    info["accepted"] = accepted
    info["ancestor"] = sample if idx is None else idx[sample]
    return th_s, l_s, logw, W, inc, info


def smc_run(y, model: Model, betas, N, step_sd, n_moves, seed, ess_frac=0.5,
            resample=True, scheme="systematic"):
    """Tempered SMC sampler from beta_0 = 0 to beta_T = 1.

    Returns a dict with theta, l, logw, W, logZ and per-step traces (ESS,
    resampled flag, accepted count)."""
    betas = np.asarray(betas, dtype=np.float64)
    T = betas.size - 1
    theta = prior_init(model, N, seed)
    l = loglik(theta, y, model)
    logw = np.zeros(N)
    W = np.full(N, 1.0 / N)
    logZ = 0.0
    tr = dict(ess=[], resampled=[], accepted=[], logZ_inc=[], u=[])
    for t in range(1, T + 1):
        theta, l, logw, W, inc, info = smc_step(theta, l, logw, y, model, betas, t, step_sd,
                                                n_moves, seed, ess_frac, resample, scheme)
        logZ += inc
        tr["ess"].append(info["ess"])
        tr["resampled"].append(info["resampled"])
        tr["accepted"].append(int(sum(int(a.sum()) for a in info["accepted"])))
        tr["logZ_inc"].append(inc)
        if info["resampled"]:
            tr["u"].append(info["u"])
    return dict(theta=theta, l=l, logw=logw, W=W, logZ=logZ, trace=tr)


# ---------------------------------------------------------------------------
# population MCMC (parallel tempering)

def exchange_pairs(M, parity, wrap):
    """Disjoint adjacent pairs (a, a+1) with a = parity mod 2; with ``wrap`` and
    parity 1 the pair (M-1, 0) closes the ring (the paper's second partition)."""
    a = np.arange(parity, M - 1, 2)
    pairs = [(int(i), int(i) + 1) for i in a]
    if wrap and parity == 1 and M >= 2 and M % 2 == 0:
        pairs.append((M - 1, 0))
    return pairs


def exchange_log_alpha(beta_a, beta_b, l_a, l_b):
    """log alpha for swapping the states of chains a and b under pi_i ~ p0 L^beta_i:
    the priors cancel, leaving (beta_a - beta_b) (l_b - l_a)."""
    return (beta_a - beta_b) * (l_b - l_a)


def pt_parity(seed, it, mode):
    if mode == "alternate":
        return it & 1
    w0, _, _, _ = px.words(seed, 0, 0, it, px.PARITY, 0)
    return int(w0) >> 31


def exchange_accepts(beta_a, beta_b, l_a, l_b, seed, it, a) -> bool:
    """The exchange decision of pair (a, b) at iteration `it`: accept iff
    log alpha >= 0 or log u < log alpha, u from the stream of the pair's first
    index a."""
    la = exchange_log_alpha(beta_a, beta_b, l_a, l_b)
    u = float(px.uniforms_open(seed, a, it, px.EXCH, 0))
    return bool(la >= 0.0 or math.log(u) < la)


def pt_exchange(theta, l, betas, parity, wrap, seed, it):
    """Exchange moves on the current partition; each pair draws its uniform from
    the stream of its first index a. Returns (theta, l, swapped pairs count)."""
    theta = np.array(theta, dtype=np.float64, copy=True)
    l = np.array(l, dtype=np.float64, copy=True)
    M = l.size
    nswap = 0
    for a, b in exchange_pairs(M, parity, wrap):
        if exchange_accepts(betas[a], betas[b], l[a], l[b], seed, it, a):
            theta[:, [a, b]] = theta[:, [b, a]]
            l[a], l[b] = l[b], l[a]
            nswap += 1
    return theta, l, nswap


def pt_iteration_pairs(theta, l, y, model: Model, betas, it, step_sd, seed, pairs):
    """One population-MCMC iteration restricted to the chains of `pairs` (pairs
    of the iteration's partition): each chain's RW-MH move at its own beta, then
    each pair's exchange. A pair depends only on its own two chains, so these
    are exactly the corresponding columns of the whole iteration.
    Returns (theta [kd][2P], l [2P], chains [2P]) with chains = (a0, b0, a1, b1, ...)."""
    betas = np.asarray(betas, dtype=np.float64)
    chains = np.array([c for p in pairs for c in p], dtype=np.int64)
    th, ll, _ = rwmh_move(np.asarray(theta)[:, chains], np.asarray(l)[chains], y, model,
                          betas[chains], step_sd, seed, it, 0, index=chains)
    for q, (a, b) in enumerate(pairs):
        if exchange_accepts(betas[a], betas[b], ll[2 * q], ll[2 * q + 1], seed, it, a):
            th[:, [2 * q, 2 * q + 1]] = th[:, [2 * q + 1, 2 * q]]
            ll[2 * q], ll[2 * q + 1] = ll[2 * q + 1], ll[2 * q]
    return th, ll, chains


def pt_run(y, model: Model, betas, iters, step_sd, seed, parity_mode="alternate",
           wrap=False, record_chain=None):
    """Population MCMC: per iteration one RW-MH move per chain at its own beta,
    then exchanges on one partition of adjacent pairs."""
    betas = np.asarray(betas, dtype=np.float64)
    M = betas.size
    theta = prior_init(model, M, seed)
    l = loglik(theta, y, model)
    acc_total = 0
    swaps = 0
    chain = []
    for it in range(iters):
        theta, l, a = rwmh_move(theta, l, y, model, betas, step_sd, seed, it, 0)
        acc_total += int(a.sum())
        parity = pt_parity(seed, it, parity_mode)
        theta, l, s = pt_exchange(theta, l, betas, parity, wrap, seed, it)
        swaps += s
        if record_chain is not None:
            chain.append(theta[:, record_chain].copy())
    return dict(theta=theta, l=l, accepted=acc_total, swaps=swaps,
                chain=np.array(chain) if chain else None)
