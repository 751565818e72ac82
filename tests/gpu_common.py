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


def loglik_threads(theta, y, model, workers=8):
    """The oracle's FP64 log-likelihood of every column of theta, the columns
    split over a thread pool (NumPy releases the GIL in its array loops). The
    arithmetic is the oracle's own; NumPy's summation blocking follows the
    array shapes, so values may differ from one call over all columns in the
    last bits (a few 1e-15 relative)."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import gmm as ogmm

    theta = np.asarray(theta, dtype=np.float64)
    N = theta.shape[1]
    parts = np.array_split(np.arange(N), max(1, min(workers, N // 256 or 1)))
    with ThreadPoolExecutor(max_workers=len(parts)) as ex:
        outs = list(ex.map(lambda ix: ogmm.loglik(theta[:, ix], y, model), parts))
    return np.concatenate(outs)


def replay_positions(N, count, seed):
    """Sorted positions for a sampled replay: `count` random ones plus the first
    and last 64 (a whole first and last tile)."""
    if N <= count + 128:
        return np.arange(N)
    rng = np.random.default_rng(seed)
    pick = rng.choice(N, size=count, replace=False)
    return np.unique(np.concatenate([pick, np.arange(64), np.arange(N - 64, N)]))
