"""Seeded synthetic inputs shared by the oracle, the tests and the bench.

This package only *generates inputs*: the observed data, the true means used to
simulate them, the inverse-temperature schedules and probe parameter values.
It holds none of the sampler's arithmetic (no likelihood, no weights, no
resampling) and it imports neither the HIP package nor the oracle, so that both
sides can consume exactly the same inputs without sharing any method code.

The random numbers that the *method* draws (proposals, accept uniforms,
resampling offsets, exchange uniforms) are not made here: each side produces
them with its own Philox4x32-10 from the published definition.
"""

from .configs import CONFIGS, WorkloadConfig, BatchedRun, batched_runs  # noqa: F401
from .data import (  # noqa: F401
    make_data,
    make_mixture_data,
    beta_schedule,
    pt_betas,
    theta_prior_draws,
    theta_near_posterior,
    lognormal_logw,
)
