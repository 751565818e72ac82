"""Sampler drivers: device-resident state plus one enqueued (or graph-replayed)
call per tempering step or PT iteration. All arithmetic runs in libsmcgpu.

SMCSampler: tempered SMC sampler (SMC Samplers and SMC Sampler subsections):
prior draws, then for t = 1..T one smc_step (reweight, ESS test and systematic
resampling on the device, RW-MH moves at beta_t). The step reads t from a
device counter and moves the population between two buffers, so two captured
hipGraphs (one per direction) are replayed alternately and the host never
waits inside the run.

BatchSampler: many independent tempered SMC runs (own data, size and seed each)
advanced together by smc_step_batched: one graph replay per tempering step for
the whole batch.

PTSampler: population MCMC with tempered chains (Population-Based MCMC
subsection): per iteration one RW-MH move per chain at its own beta, then
exchange moves on one partition of adjacent pairs.

The mixture samplers hold their own device copy of the data; 1-D data are
sorted into ascending order once, on the device (smc_sort_data), which leaves
the likelihood unchanged up to rounding and lets the FP32 likelihood take its
pivot form.
"""

from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np
import torch

from .api import (Batch, Context, Gmm, Graph, fsv_init, fsv_step, fsv_steps, pt_iteration,
                  pt_iterations, pt_record, smc_loglik, smc_prior_init, smc_sort_data,
                  smc_step, smc_step_batched, smc_steps)


def _dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).cuda()


class SMCSampler:
    def __init__(self, ctx: Context, model: Gmm, y, N: int, betas, step_sd: float,
                 n_moves: int, seed: int, ess_frac: float = 0.5, prec: str = "fp32",
                 stream: Optional[torch.cuda.Stream] = None, scheme: str = "systematic"):
        self.ctx, self.model, self.N = ctx, model, int(N)
        self.step_sd, self.n_moves, self.seed = float(step_sd), int(n_moves), int(seed)
        self.ess_frac, self.prec, self.scheme = float(ess_frac), prec, scheme
        self.T = len(betas) - 1
        self.stream = stream or torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            self.y = _dev(y, torch.float32)
            if model.d == 1:
                smc_sort_data(self.y, stream=self.stream)
            self.beta = _dev(np.asarray(betas, dtype=np.float64), torch.float64)
            kd = model.kd
            self.thetas = [torch.empty((kd, self.N), dtype=torch.float64, device="cuda")
                           for _ in range(2)]
            self.logliks = [torch.empty(self.N, dtype=torch.float64, device="cuda")
                            for _ in range(2)]
            self.logw = torch.zeros(self.N, dtype=torch.float64, device="cuda")
            self.W = torch.full((self.N,), 1.0 / self.N, dtype=torch.float64, device="cuda")
            self.t = torch.ones(1, dtype=torch.int32, device="cuda")
            self.stats = torch.zeros(4, dtype=torch.float64, device="cuda")
            self.n_accept = torch.zeros(1, dtype=torch.int64, device="cuda")
        ctx.reserve(self.N, model.kd, self.y.shape[0] if prec == "bf16x3" else 0)
        self.cur = 0                       # buffer holding the current population
        self.graphs: dict = {}             # (start buffer, steps) -> Graph

    @property
    def theta(self) -> torch.Tensor:
        return self.thetas[self.cur]

    @property
    def loglik(self) -> torch.Tensor:
        return self.logliks[self.cur]

    def init(self):
        """theta_0 from the prior, l(theta_0), logw = 0, t = 1, statistics cleared."""
        self.cur = 0
        with torch.cuda.stream(self.stream):
            smc_prior_init(self.ctx, self.model, self.N, self.seed, out=self.thetas[0],
                           stream=self.stream)
            smc_loglik(self.ctx, self.model, self.y, self.thetas[0], self.prec,
                       out=self.logliks[0], stream=self.stream)
            self.logw.zero_()
            self.W.fill_(1.0 / self.N)
            self.t.fill_(1)
            self.stats.zero_()
            self.n_accept.zero_()

    def enqueue_step(self, src: int):
        dst = 1 - src
        self.ctx.set_resampling(self.scheme)
        smc_step(self.ctx, self.model, self.y, self.thetas[src], self.logliks[src],
                 self.thetas[dst], self.logliks[dst], self.logw, self.W, self.beta, self.t,
                 self.step_sd, self.n_moves, self.seed, self.ess_frac, self.prec, self.stats,
                 self.n_accept, stream=self.stream)

    def enqueue_steps(self, src: int, steps: int):
        """`steps` consecutive steps from buffer `src` in one smc_steps call (each
        move after the first step's also makes the next step's reweight)."""
        self.ctx.set_resampling(self.scheme)
        smc_steps(self.ctx, self.model, self.y, self.thetas[src], self.logliks[src],
                  self.thetas[1 - src], self.logliks[1 - src], self.logw, self.W, self.beta,
                  self.t, steps, self.step_sd, self.n_moves, self.seed, self.ess_frac, self.prec,
                  self.stats, self.n_accept, stream=self.stream)

    def capture(self, src: Optional[int] = None, steps: int = 1) -> Graph:
        """The hipGraph of `steps` consecutive tempering steps starting from buffer
        `src` (replayable for every t: t, beta_t and the resampling decision live
        on the device). An even number of steps ends on the buffer it started from."""
        src = self.cur if src is None else src
        key = (src, int(steps))
        if key not in self.graphs:
            g = Graph(self.ctx, self.stream)
            with g:
                self.enqueue_steps(src, int(steps))
            self.graphs[key] = g
        return self.graphs[key]

    def step(self, graph: bool = True, steps: int = 1):
        """Advance `steps` tempering steps in one smc_steps call (replayed as one
        graph when graph=True); a single step is exactly an smc_step call."""
        if graph:
            self.capture(self.cur, steps).launch()
        elif int(steps) == 1:
            self.enqueue_step(self.cur)
        else:
            self.enqueue_steps(self.cur, int(steps))
        self.cur = self.cur ^ (int(steps) & 1)

    def advance(self, steps: int, graph: bool = True, steps_per_graph: int = 10):
        """Advance `steps` steps in groups of `steps_per_graph` (the last group
        holds the remainder), each group one graph replay (graph=True) or one
        eager smc_steps call; the same grouping gives the same results either way."""
        u = max(1, int(steps_per_graph))
        for _ in range(steps // u):
            self.step(graph, u)
        if steps % u:
            self.step(graph, steps % u)

    def run(self, graph: bool = True, steps: Optional[int] = None, steps_per_graph: int = 1):
        self.init()
        self.advance(self.T if steps is None else steps, graph, steps_per_graph)
        self.stream.synchronize()
        self.ctx.check(self.stream)
        return self.results()

    def results(self):
        self.stream.synchronize()
        st = self.stats.cpu().numpy()
        return dict(logZ=float(st[0]), ess=float(st[1]), resamples=int(st[2]),
                    accepted=int(self.n_accept.cpu().item()), t=int(self.t.cpu().item()),
                    theta=self.theta.cpu().numpy(), l=self.loglik.cpu().numpy(),
                    logw=self.logw.cpu().numpy(), W=self.W.cpu().numpy())


class PTSampler:
    def __init__(self, ctx: Context, model: Gmm, y, betas, step_sd: float, seed: int,
                 parity_mode: int = 0, wrap: bool = False, prec: str = "fp32",
                 stream: Optional[torch.cuda.Stream] = None, record_chain: Optional[int] = None,
                 record_iters: int = 0, fused_iterations: bool = True):
        self.ctx, self.model = ctx, model
        self.M = len(betas)
        self.fused = bool(fused_iterations)
        self.step_sd, self.seed = float(step_sd), int(seed)
        self.parity_mode, self.wrap, self.prec = int(parity_mode), bool(wrap), prec
        self.stream = stream or torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            self.y = _dev(y, torch.float32)
            if model.d == 1:
                smc_sort_data(self.y, stream=self.stream)
            self.beta = _dev(np.asarray(betas, dtype=np.float64), torch.float64)
            self.theta = torch.empty((model.kd, self.M), dtype=torch.float64, device="cuda")
            self.loglik = torch.empty(self.M, dtype=torch.float64, device="cuda")
            self.it = torch.zeros(1, dtype=torch.int32, device="cuda")
            self.n_accept = torch.zeros(1, dtype=torch.int64, device="cuda")
            self.n_swap = torch.zeros(1, dtype=torch.int32, device="cuda")
        ctx.reserve(self.M, model.kd, self.y.shape[0] if prec == "bf16x3" else 0)
        self.graphs: Dict[int, Graph] = {}
        self.record_chain = record_chain
        self.record = (torch.zeros((int(record_iters), model.kd), dtype=torch.float64,
                                   device="cuda") if record_chain is not None else None)

    def init(self):
        with torch.cuda.stream(self.stream):
            smc_prior_init(self.ctx, self.model, self.M, self.seed, out=self.theta,
                           stream=self.stream)
            smc_loglik(self.ctx, self.model, self.y, self.theta, self.prec, out=self.loglik,
                       stream=self.stream)
            self.it.zero_()
            self.n_accept.zero_()
            self.n_swap.zero_()

    def enqueue_iteration(self):
        pt_iteration(self.ctx, self.model, self.y, self.theta, self.loglik, self.beta, self.it,
                     self.step_sd, self.seed, self.parity_mode, self.wrap, self.prec,
                     self.n_accept, self.n_swap, stream=self.stream)
        if self.record is not None:
            pt_record(self.ctx, self.theta, self.record_chain, self.it, self.record,
                      stream=self.stream)

    def enqueue_iterations(self, count: int):
        """`count` iterations: one pt_iterations call (a single launch for small
        populations) unless the target chain is recorded after every iteration
        or the sampler was made with fused_iterations=False."""
        if self.record is not None or not self.fused:
            for _ in range(count):
                self.enqueue_iteration()
            return
        pt_iterations(self.ctx, self.model, self.y, self.theta, self.loglik, self.beta, self.it,
                      count, self.step_sd, self.seed, self.parity_mode, self.wrap, self.prec,
                      self.n_accept, self.n_swap, stream=self.stream)

    def capture(self, iterations: int = 1) -> Graph:
        """A graph of `iterations` consecutive iterations (the iteration index
        lives on the device, so one graph serves every position in the run)."""
        g = self.graphs.get(iterations)
        if g is None:
            g = Graph(self.ctx, self.stream)
            with g:
                self.enqueue_iterations(iterations)
            self.graphs[iterations] = g
        return g

    def advance(self, iterations: int, graph: bool = True, iters_per_graph: int = 1):
        done = 0
        while done < iterations:
            c = min(int(iters_per_graph), iterations - done)
            if graph:
                self.capture(c).launch()
            else:
                self.enqueue_iterations(c)
            done += c

    def run(self, iterations: int, graph: bool = True, iters_per_graph: int = 1):
        self.init()
        self.advance(iterations, graph, iters_per_graph)
        self.stream.synchronize()
        self.ctx.check(self.stream)
        return self.results()

    def results(self):
        self.stream.synchronize()
        return dict(theta=self.theta.cpu().numpy(), l=self.loglik.cpu().numpy(),
                    accepted=int(self.n_accept.cpu().item()),
                    swaps=int(self.n_swap.cpu().item()), it=int(self.it.cpu().item()),
                    chain=None if self.record is None else self.record.cpu().numpy())


class BatchSampler:
    def __init__(self, ctx: Context, model: Gmm, datas, Ns, seeds, betas, step_sd: float,
                 n_moves: int, ess_frac: float = 0.5, prec: str = "fp32",
                 stream: Optional[torch.cuda.Stream] = None, scheme: str = "systematic"):
        if model.d != 1:
            raise ValueError("batched runs are one-dimensional mixtures")
        self.ctx, self.model, self.scheme = ctx, model, scheme
        self.Ns = [int(x) for x in Ns]
        self.ns = [int(np.asarray(y).size) for y in datas]
        self.seeds = [int(x) for x in seeds]
        self.R = len(self.Ns)
        self.p_off = np.concatenate([[0], np.cumsum(self.Ns)[:-1]]).astype(np.int64)
        self.y_off = np.concatenate([[0], np.cumsum(self.ns)[:-1]]).astype(np.int64)
        self.N_total = int(sum(self.Ns))
        self.step_sd, self.n_moves = float(step_sd), int(n_moves)
        self.ess_frac, self.prec = float(ess_frac), prec
        self.T = len(betas) - 1
        self.stream = stream or torch.cuda.Stream()
        kd = model.kd
        with torch.cuda.stream(self.stream):
            self.y = _dev(np.concatenate([np.asarray(y, dtype=np.float32).ravel() for y in datas]),
                          torch.float32)
            for r in range(self.R):                  # each run's data in ascending order
                smc_sort_data(self.y[self.y_off[r]:self.y_off[r] + self.ns[r]], stream=self.stream)
            self.beta = _dev(np.asarray(betas, dtype=np.float64), torch.float64)
            self.theta = torch.empty(kd * self.N_total, dtype=torch.float64, device="cuda")
            self.loglik = torch.empty(self.N_total, dtype=torch.float64, device="cuda")
            self.logw = torch.zeros(self.N_total, dtype=torch.float64, device="cuda")
            self.W = torch.empty(self.N_total, dtype=torch.float64, device="cuda")
            self.t = torch.ones(1, dtype=torch.int32, device="cuda")
            self.stats = torch.zeros(4 * self.R, dtype=torch.float64, device="cuda")
            self.n_accept = torch.zeros(1, dtype=torch.int64, device="cuda")
        self.batch = Batch(ctx, [(self.p_off[r], self.y_off[r], self.Ns[r], self.ns[r],
                                  self.seeds[r]) for r in range(self.R)], kd)
        ctx.reserve(max(self.Ns), kd)
        self.graph: Optional[Graph] = None

    def theta_of(self, r: int) -> torch.Tensor:
        kd = self.model.kd
        a = kd * int(self.p_off[r])
        return self.theta[a:a + kd * self.Ns[r]].view(kd, self.Ns[r])

    def _slice(self, t: torch.Tensor, r: int) -> torch.Tensor:
        a = int(self.p_off[r])
        return t[a:a + self.Ns[r]]

    def init(self):
        with torch.cuda.stream(self.stream):
            for r in range(self.R):
                smc_prior_init(self.ctx, self.model, self.Ns[r], self.seeds[r],
                               out=self.theta_of(r), stream=self.stream)
                a = int(self.y_off[r])
                smc_loglik(self.ctx, self.model, self.y[a:a + self.ns[r]], self.theta_of(r),
                           self.prec, out=self._slice(self.loglik, r), stream=self.stream)
            self.logw.zero_()
            self.t.fill_(1)
            self.stats.zero_()
            self.n_accept.zero_()

    def enqueue_step(self):
        self.ctx.set_resampling(self.scheme)
        smc_step_batched(self.ctx, self.batch, self.model, self.y, self.theta, self.loglik,
                         self.logw, self.W, self.beta, self.t, self.step_sd, self.n_moves,
                         self.ess_frac, self.prec, self.stats, self.n_accept, stream=self.stream)

    def capture(self) -> Graph:
        if self.graph is None:
            g = Graph(self.ctx, self.stream)
            with g:
                self.enqueue_step()
            self.graph = g
        return self.graph

    def run(self, graph: bool = True, steps: Optional[int] = None):
        self.init()
        for _ in range(self.T if steps is None else steps):
            if graph:
                self.capture().launch()
            else:
                self.enqueue_step()
        self.stream.synchronize()
        self.ctx.check(self.stream)
        return self.results()

    def results(self):
        self.stream.synchronize()
        st = self.stats.cpu().numpy().reshape(self.R, 4)
        return dict(logZ=st[:, 0].copy(), ess=st[:, 1].copy(), resamples=st[:, 2].astype(int),
                    accepted=int(self.n_accept.cpu().item()), t=int(self.t.cpu().item()),
                    theta=[self.theta_of(r).cpu().numpy() for r in range(self.R)],
                    l=[self._slice(self.loglik, r).cpu().numpy() for r in range(self.R)])


def mode_census(theta, W=None):
    """Weight of each of the k! symmetric posterior modes (Mixture Modelling:
    with exchangeable priors the posterior of the k means is invariant to
    relabelling). A 1-D particle belongs to the mode given by the ranks of its k
    means. theta: [k][N] (tensor or array); W: normalised weights (None: equal).
    Returns {rank tuple: weight share}, the shares summing to one. Host-side
    analysis of a finished run; nothing here is on the sampling path."""
    th = theta.detach().cpu().numpy() if isinstance(theta, torch.Tensor) else np.asarray(theta)
    k, N = th.shape
    w = (np.full(N, 1.0 / N) if W is None else
         (W.detach().cpu().numpy() if isinstance(W, torch.Tensor) else np.asarray(W, float)))
    ranks = np.argsort(np.argsort(th, axis=0, kind="stable"), axis=0, kind="stable")
    code = np.zeros(N, dtype=np.int64)
    for c in range(k):
        code = code * k + ranks[c]
    shares = np.bincount(code, weights=w, minlength=k ** k)
    out = {}
    for v in np.nonzero(shares)[0]:
        digits, x = [], int(v)
        for _ in range(k):
            digits.append(x % k)
            x //= k
        out[tuple(reversed(digits))] = float(shares[v])
    return out


def traversal_time(chain) -> Optional[int]:
    """Iterations until a recorded chain has visited all k! symmetric modes
    (Population-Based MCMC subsection); chain: [iterations, k] of 1-D means.
    None if some mode was never visited."""
    ch = np.asarray(chain)
    k = ch.shape[1]
    ranks = np.argsort(np.argsort(ch, axis=1, kind="stable"), axis=1, kind="stable")
    code = np.zeros(ch.shape[0], dtype=np.int64)
    for c in range(k):
        code = code * k + ranks[:, c]
    seen = set()
    need = math.factorial(k)
    for t, v in enumerate(code):
        seen.add(int(v))
        if len(seen) == need:
            return t + 1
    return None


class FSVFilter:
    """Bootstrap particle filter of the factor stochastic-volatility model over
    observations y [T, m]; the step index lives on the device, so a graph of
    several steps replays anywhere in the run."""

    def __init__(self, ctx: Context, model, y, N: int, seed: int, ess_frac: float = 0.5,
                 stream: Optional[torch.cuda.Stream] = None, scheme: str = "systematic"):
        self.ctx, self.model, self.N, self.seed = ctx, model, int(N), int(seed)
        self.ess_frac, self.scheme = float(ess_frac), scheme
        self.k = len(model.phi)
        self.stream = stream or torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            self.y = _dev(np.asarray(y, dtype=np.float64), torch.float64)
            self.T = int(self.y.shape[0])
            self.x = torch.zeros((self.k, self.N), dtype=torch.float64, device="cuda")
            self.x_tmp = torch.empty_like(self.x)
            self.logw = torch.zeros(self.N, dtype=torch.float64, device="cuda")
            self.t = torch.ones(1, dtype=torch.int32, device="cuda")
            self.stats = torch.zeros(4, dtype=torch.float64, device="cuda")
            self.moments = torch.zeros((self.T, 2 * self.k), dtype=torch.float64, device="cuda")
        ctx.reserve(self.N, self.k)
        self.graphs: Dict[int, Graph] = {}

    def init(self):
        with torch.cuda.stream(self.stream):
            fsv_init(self.ctx, self.x, self.logw, stream=self.stream)
            self.t.fill_(1)
            self.stats.zero_()

    def enqueue_step(self):
        self.ctx.set_resampling(self.scheme)
        fsv_step(self.ctx, self.model, self.y, self.x, self.x_tmp, self.logw, self.t, self.seed,
                 self.ess_frac, self.stats, self.moments, stream=self.stream)

    def enqueue_steps(self, steps: int):
        """`steps` consecutive steps in one fsv_steps call (each propagation
        takes the previous step's resampling itself)."""
        self.ctx.set_resampling(self.scheme)
        fsv_steps(self.ctx, self.model, self.y, self.x, self.x_tmp, self.logw, self.t, steps,
                  self.seed, self.ess_frac, self.stats, self.moments, stream=self.stream)

    def capture(self, steps: int = 1) -> Graph:
        g = self.graphs.get(steps)
        if g is None:
            g = Graph(self.ctx, self.stream)
            with g:
                self.enqueue_steps(steps)
            self.graphs[steps] = g
        return g

    def advance(self, steps: int, graph: bool = True, steps_per_graph: int = 1,
                chained: bool = True):
        """Groups of `steps_per_graph` steps, each one graph replay (graph=True)
        or one eager call: fsv_steps, or (chained=False) single fsv_step calls."""
        done = 0
        while done < steps:
            c = min(int(steps_per_graph), steps - done)
            if graph:
                self.capture(c).launch()
            elif chained:
                self.enqueue_steps(c)
            else:
                for _ in range(c):
                    self.enqueue_step()
            done += c

    def run(self, graph: bool = True, steps_per_graph: int = 1, chained: bool = True):
        self.init()
        self.advance(self.T, graph, steps_per_graph, chained)
        self.stream.synchronize()
        self.ctx.check(self.stream)
        return self.results()

    def results(self):
        self.stream.synchronize()
        st = self.stats.cpu().numpy()
        mom = self.moments.cpu().numpy()
        return dict(loglik=float(st[0]), ess=float(st[1]), resamples=int(st[2]),
                    mean=mom[:, :self.k], sd=mom[:, self.k:], x=self.x.cpu().numpy(),
                    logw=self.logw.cpu().numpy(), t=int(self.t.cpu().item()))
