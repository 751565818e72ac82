"""Shared helpers of the GPU parity tests (imported by tests only)."""

import numpy as np

from oracle.gmm import Model


def oracle_model(g):
    """The oracle's Model for a binding Gmm (same parameters, no shared code)."""
    return Model(k=g.k, d=g.d, sigma2=g.sigma2, log_w=tuple(g.log_w), prior=g.prior,
                 prior_a=g.prior_a, prior_b=g.prior_b)


def rel_err(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return np.abs(got - want) / np.maximum(np.abs(want), 1e-300)


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
