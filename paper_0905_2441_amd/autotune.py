"""Launch-shape autotuner for the likelihood kernels.

The tunable is the number of data slices per 64-particle tile: how many waves
(and, above 16, how many workgroups) share one tile's observations. It trades
the per-wave fixed work (proposal normals, accept test, partial-sum combine)
against filling the 256 CUs and balancing the waves over each CU's four SIMDs.
For each (k, d, n, N, precision) shape the tuner times one RW-MH move per
candidate on the device, with HIP events on its own stream, and keeps the
fastest; the result is a list of launch rules for ``Context.set_launch_table``
(C ABI ``smc_set_launch_table``), which can be saved as JSON and reloaded.

Batched runs (``tune_batched``): the persistent move gives every tile of a run
S of its workgroup's 8 waves (so 8 / S tiles share a workgroup). For each
power-of-two range of n among the runs, the tuner times graph-replayed batched
steps of just those runs for S = 1, 2, 4, 8 and keeps the fastest, giving one
batch rule per range.

Usage: python -m paper_0905_2441_amd.autotune --shape 4,1,1000,131072,fp32 [--out table.json]
"""

from __future__ import annotations

import argparse
import json
import math
from typing import Dict, Iterable, List, Optional, Sequence

import numpy as np
import torch

from .api import Context, Gmm, smc_rwmh_move, smc_sort_data

# Slice counts tried: 1..4 for short data, then multiples of 4 so that every
# SIMD of a CU receives the same number of waves of a workgroup.
CANDIDATES = (1, 2, 3, 4, 8, 12, 16, 24, 32, 48, 64, 96, 128)
SPLIT_CAP = 32768          # largest N whose tiles may span several workgroups
MIN_PER_SLICE = 8          # observations per slice below which a candidate is skipped


def candidates(n: int, N: int, prec: str = "fp32") -> List[int]:
    top = 16 if (prec == "bf16x3" or N > SPLIT_CAP) else CANDIDATES[-1]
    out = [T for T in CANDIDATES if T <= top and T <= n and n // T >= MIN_PER_SLICE]
    return out or [1]


def time_move(ctx: Context, model: Gmm, y, theta, loglik, prec: str, reps: int,
              stream: torch.cuda.Stream) -> float:
    """Mean device time (ms) of one RW-MH move over `reps` back-to-back moves."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for i in range(2):                      # warm the code object and caches
        smc_rwmh_move(ctx, model, y, theta, loglik, 1.0, 0.1, 1, i, 0, prec, stream=stream)
    e0.record(stream)
    for i in range(reps):
        smc_rwmh_move(ctx, model, y, theta, loglik, 1.0, 0.1, 1, 2 + i, 0, prec, stream=stream)
    e1.record(stream)
    e1.synchronize()
    ctx.check(stream)
    return e0.elapsed_time(e1) / reps


def tune_shape(ctx: Context, k: int, d: int, n: int, N: int, prec: str = "fp32",
               reps: int = 20, cands: Optional[Sequence[int]] = None, seed: int = 0) -> dict:
    """Time every candidate slice count for one shape; returns
    {"best": T, "ms": {T: ms}}. Inputs are synthetic: standard-normal data
    (1-D data in ascending order, as the samplers hold them, so that the FP32
    likelihood takes its pivot form) and standard-normal means. The kernels'
    time depends on the values only through the FP32 form a wave takes and,
    in the pivot form, through how many components it evaluates."""
    model = Gmm.equal_weights(k, d, 1.0)
    stream = torch.cuda.Stream()
    gen = torch.Generator(device="cuda").manual_seed(seed)
    with torch.cuda.stream(stream):
        y = torch.randn((n, d) if d > 1 else (n,), generator=gen, device="cuda",
                        dtype=torch.float32)
        if d == 1:
            smc_sort_data(y, stream=stream)
        theta = torch.randn((k * d, N), generator=gen, device="cuda", dtype=torch.float64)
        loglik = torch.full((N,), -1.0e6, device="cuda", dtype=torch.float64)
    ctx.reserve(N, k * d, n if prec == "bf16x3" else 0)
    times: Dict[int, float] = {}
    try:
        for T in (cands or candidates(n, N, prec)):
            ctx.set_slices(T)
            times[T] = time_move(ctx, model, y, theta, loglik, prec, reps, stream)
    finally:
        ctx.set_slices(0)
    best = min(times, key=times.get)
    return {"best": best, "ms": times}


def bucket(v: int) -> tuple:
    """The power-of-two range [2^e, 2^(e+1) - 1] that holds v."""
    e = int(math.floor(math.log2(max(1, v))))
    return 1 << e, (1 << (e + 1)) - 1


def make_rules(ctx: Context, shapes: Iterable[tuple], reps: int = 20, exact: bool = False,
               log=None) -> List[dict]:
    """Tune each (k, d, n, N, prec) shape and return one rule per shape, valid
    for that exact shape or (default) for its power-of-two buckets of n and N."""
    rules = []
    for (k, d, n, N, prec) in shapes:
        r = tune_shape(ctx, k, d, n, N, prec, reps)
        n_lo, n_hi = (n, n) if exact else bucket(n)
        N_lo, N_hi = (N, N) if exact else bucket(N)
        rules.append(dict(k=k, d=d, prec=prec, slices=r["best"], n_lo=n_lo, n_hi=n_hi,
                          N_lo=N_lo, N_hi=N_hi,
                          ms={str(t): round(v, 5) for t, v in r["ms"].items()}))
        if log:
            log(f"[autotune] k={k} d={d} n={n} N={N} {prec}: slices {r['best']} "
                f"({r['ms'][r['best']]:.4f} ms/move; "
                + ", ".join(f"{t}: {v:.4f}" for t, v in r["ms"].items()) + ")")
    return rules


BATCH_CANDIDATES = (1, 2, 4, 8)


def time_batched_step(ctx: Context, model: Gmm, datas, Ns, seeds, betas, step_sd: float,
                      n_moves: int, ess_frac: float, prec: str, reps: int) -> float:
    """Mean device time (ms) of one graph-replayed batched step of these runs
    under the context's current launch table: the runs start from the prior,
    one step warms the graph, then `reps` steps are timed with HIP events."""
    from .samplers import BatchSampler
    b = BatchSampler(ctx, model, datas, Ns, seeds, betas, step_sd, n_moves, ess_frac=ess_frac,
                     prec=prec)
    try:
        b.init()
        g = b.capture()
        g.launch()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(b.stream)
        for _ in range(reps):
            g.launch()
        e1.record(b.stream)
        e1.synchronize()
        ctx.check(b.stream)
        return e0.elapsed_time(e1) / reps
    finally:
        if b.graph is not None:
            b.graph.close()
        b.batch.close()


def tune_batched(ctx: Context, model: Gmm, datas, Ns, seeds, betas, step_sd: float,
                 n_moves: int, ess_frac: float = 0.5, prec: str = "fp32", reps: int = 3,
                 log=None) -> List[dict]:
    """Batch rules (kind "batch") for the runs' power-of-two ranges of n: for
    each range, graph-replayed batched steps of the runs in it are timed with
    every S in BATCH_CANDIDATES and the fastest is kept. Other rules of the
    context's table are kept while tuning and the batch rules are returned (the
    caller installs them)."""
    base = [r for r in ctx.rules if r.get("kind", "call") != "batch"]
    ns = [int(np.asarray(y).size) for y in datas]
    buckets = sorted({bucket(n) for n in ns})
    out = []
    for lo, hi in buckets:
        sel = [i for i, n in enumerate(ns) if lo <= n <= hi]
        times = {}
        for S in BATCH_CANDIDATES:
            rule = dict(k=model.k, d=1, prec=prec, kind="batch", slices=S, n_lo=lo, n_hi=hi,
                        N_lo=1, N_hi=(1 << 31) - 1)
            ctx.set_launch_table(list(base) + [rule])
            times[S] = time_batched_step(ctx, model, [datas[i] for i in sel],
                                         [Ns[i] for i in sel], [seeds[i] for i in sel], betas,
                                         step_sd, n_moves, ess_frac, prec, reps)
        best = min(times, key=times.get)
        out.append(dict(k=model.k, d=1, prec=prec, kind="batch", slices=best, n_lo=lo, n_hi=hi,
                        N_lo=1, N_hi=(1 << 31) - 1, runs=len(sel),
                        ms={str(t): round(v, 4) for t, v in times.items()}))
        if log:
            log(f"[autotune] batch n in [{lo}, {hi}] ({len(sel)} runs): S = {best} "
                f"({', '.join(f'{t}: {v:.3f}' for t, v in times.items())} ms/step)")
    ctx.set_launch_table(list(base))
    return out


def save(rules: Sequence[dict], path: str) -> None:
    with open(path, "w") as f:
        json.dump({"rules": list(rules)}, f, indent=1)


def load(ctx: Context, path: str) -> List[dict]:
    with open(path) as f:
        rules = json.load(f)["rules"]
    ctx.set_launch_table(rules)
    return rules


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--shape", action="append", required=True,
                    help="k,d,n,N,prec (repeatable)")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--exact", action="store_true", help="rules for the exact shapes only")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    shapes = []
    for s in a.shape:
        k, d, n, N, prec = s.split(",")
        shapes.append((int(k), int(d), int(n), int(N), prec))
    ctx = Context(0)
    rules = make_rules(ctx, shapes, a.reps, a.exact, log=print)
    if a.out:
        save(rules, a.out)
    print(json.dumps({"rules": rules}))


if __name__ == "__main__":
    main()
