"""The five workloads the sampler is exercised on.

Model (Mixture Modelling section of the paper): a univariate (or d-variate,
identity-covariance) Gaussian mixture with k components, known equal weights
and known variance, unknown means. The paper's own settings are k = 4,
sigma = 0.55, w = 1/4, m = 100 observations simulated at means (-3, 0, 3, 6),
a uniform prior on [-10, 10]^k and tempering schedules (t/M)^2. The five
workloads below scale that model up; the paper's settings remain reachable
through the ``paper_mode`` helper.

Every workload is synthetic, as are the paper's own (the data are simulated
from the mixture).
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class WorkloadConfig:
    name: str
    k: int
    d: int
    n: int                      # observations
    N: int                      # particles (SMC) or chains (PT)
    sigma2: float               # known component variance
    true_means: Optional[Tuple[float, ...]]   # None: drawn from the data seed
    data_seed: int
    run_seed: int
    T: int                      # tempering steps (SMC) or iterations (PT)
    schedule: str               # "linear", "quadratic", "pt_quartic", ...
    step_sd: float              # random-walk proposal standard deviation
    n_moves: int                # RW-MH moves per tempering step
    prior: str = "gauss"        # "gauss" (mean prior_a, sd prior_b) or "box" [prior_a, prior_b]
    prior_a: float = 0.0
    prior_b: float = 10.0
    ess_frac: float = 0.5       # resample when ESS < ess_frac * N
    sampler: str = "smc"        # "smc" or "pt"
    precisions: Tuple[str, ...] = ("fp64",)
    true_mean_sd: float = 0.0   # for drawn true means (d-dim workload)

    @property
    def log_w(self) -> Tuple[float, ...]:
        return tuple([math.log(1.0 / self.k)] * self.k)


CONFIGS = {
    # Plain FP64 SMC sampler, small: the configuration the oracle finishes in seconds.
    "gmm1d_k4_n100_N1024": WorkloadConfig(
        name="gmm1d_k4_n100_N1024", k=4, d=1, n=100, N=1024, sigma2=0.55,
        true_means=(-3.0, 0.0, 3.0, 6.0), data_seed=1, run_seed=101, T=50,
        schedule="linear", step_sd=0.5, n_moves=1, precisions=("fp64",)),
    # The same model at scale: the headline workload.
    "gmm1d_k4_n1000_N131072": WorkloadConfig(
        name="gmm1d_k4_n1000_N131072", k=4, d=1, n=1000, N=131072, sigma2=0.55,
        true_means=(-3.0, 0.0, 3.0, 6.0), data_seed=2, run_seed=102, T=100,
        schedule="quadratic", step_sd=0.5, n_moves=1, precisions=("fp32", "fp64")),
    # Population MCMC (parallel tempering) with many chains and long data.
    "pt_k4_n10000_M8192": WorkloadConfig(
        name="pt_k4_n10000_M8192", k=4, d=1, n=10000, N=8192, sigma2=0.55,
        true_means=(-3.0, 0.0, 3.0, 6.0), data_seed=3, run_seed=103, T=5000,
        schedule="pt_quartic", step_sd=0.5, n_moves=1, sampler="pt",
        precisions=("fp32",)),
    # d-dimensional mixture: 8 components in 8 dimensions, identity covariance.
    "gmm8d_k8_n65536_N16384": WorkloadConfig(
        name="gmm8d_k8_n65536_N16384", k=8, d=8, n=65536, N=16384, sigma2=1.0,
        true_means=None, true_mean_sd=3.0, data_seed=4, run_seed=104, T=100,
        schedule="quadratic", step_sd=0.5, n_moves=1,
        precisions=("bf16x3", "fp64")),
}


@dataclasses.dataclass(frozen=True)
class BatchedRun:
    index: int
    n: int
    N: int
    true_means: Tuple[float, ...]
    data_seed: int
    run_seed: int


def batched_runs(R: int = 256, master_seed: int = 5000) -> List[BatchedRun]:
    """Batched serving-style workload: R independent 1-D k = 4 runs.

    Run r has its own seed (master_seed + r); its n is log-uniform on
    [100, 100000], its N is drawn from {1024, 4096, 16384, 65536} and its four
    true means are uniform on [-6, 9]. Schedule, proposal sd and prior are the
    headline workload's (100 quadratic steps, sd 0.5, N(0, 10^2)).
    """
    runs = []
    for r in range(R):
        seed = master_seed + r
        rng = np.random.Generator(np.random.PCG64(seed))
        n = int(round(math.exp(rng.uniform(math.log(100.0), math.log(1.0e5)))))
        N = int(rng.choice([1024, 4096, 16384, 65536]))
        means = tuple(float(x) for x in rng.uniform(-6.0, 9.0, size=4))
        runs.append(BatchedRun(index=r, n=n, N=N, true_means=means,
                               data_seed=seed, run_seed=seed))
    return runs


BATCHED = dict(k=4, d=1, sigma2=0.55, T=100, schedule="quadratic", step_sd=0.5,
               n_moves=1, prior="gauss", prior_a=0.0, prior_b=10.0, ess_frac=0.5)


def paper_mode(N: int = 8192) -> WorkloadConfig:
    """The paper's own SMC-sampler settings (SMC Sampler subsection).

    sigma = 0.55 read as a standard deviation (variance 0.3025), uniform prior on
    [-10, 10]^4, 200 steps of (t/200)^2, ten N(0, I) random-walk moves per step,
    m = 100 observations at means (-3, 0, 3, 6).
    """
    return WorkloadConfig(
        name=f"paper_smc_N{N}", k=4, d=1, n=100, N=N, sigma2=0.55 ** 2,
        true_means=(-3.0, 0.0, 3.0, 6.0), data_seed=1, run_seed=201, T=200,
        schedule="quadratic", step_sd=1.0, n_moves=10, prior="box",
        prior_a=-10.0, prior_b=10.0, precisions=("fp32", "fp64"))
