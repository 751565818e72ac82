"""GPU parity of the factor stochastic-volatility particle filter against the
FP64 oracle on the same seeded observations and Philox streams."""

import numpy as np
import pytest
import torch

from gpu_common import announce
from oracle import fsv as ofsv
from workloads.fsv import PAPER_FSV, FsvModel, simulate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smc():
    import paper_0905_2441_amd as smc
    return smc


@pytest.fixture(scope="module")
def ctx(smc):
    return smc.Context(0)


def _compare(r, ref, N):
    assert r["resamples"] == int(ref["resampled"].sum())
    assert abs(r["loglik"] - ref["loglik"]) <= 1e-9 * max(1.0, abs(ref["loglik"]))
    assert np.max(np.abs(r["mean"] - ref["mean"])) <= 1e-9
    assert np.max(np.abs(r["sd"] - ref["sd"])) <= 1e-8
    assert np.max(np.abs(r["x"] - ref["x_end"])) <= 1e-11
    assert np.max(np.abs(r["logw"] - ref["logw_end"])) <= 1e-9 * max(1.0, np.abs(ref["logw_end"]).max())


@pytest.mark.parametrize("N,graph", [(1000, False), (1000, True), (1, False), (4097, True)])
def test_fsv_paper_model_matches_oracle(smc, ctx, N, graph):
    announce(f"fsv paper model N={N} graph={graph}")
    _, y = simulate(PAPER_FSV, 40, 11)
    f = smc.FSVFilter(ctx, PAPER_FSV, y, N, seed=5)
    r = f.run(graph=graph, steps_per_graph=7)
    assert r["t"] == 41
    ref = ofsv.particle_filter(y, PAPER_FSV, N, 5)
    _compare(r, ref, N)


@pytest.mark.parametrize("model", [FsvModel(B=((1.1,),), psi=(0.5,), phi=(0.9,), U=((0.5,),)),
                                   FsvModel(B=((1.0, 0.0), (0.4, 0.8)), psi=(0.3, 0.6),
                                            phi=(0.95, 0.8), U=((0.4, 0.1), (0.1, 0.3)))])
def test_fsv_small_models_match_oracle(smc, ctx, model):
    announce(f"fsv m={model.m} k={model.k}")
    _, y = simulate(model, 30, 3)
    r = smc.FSVFilter(ctx, model, y, 2000, seed=8).run(graph=True, steps_per_graph=10)
    _compare(r, ofsv.particle_filter(y, model, 2000, 8), 2000)


def test_fsv_paper_length_run(smc, ctx):
    """T = 200 observations, N = 16384 particles, as in the paper's runs."""
    announce("fsv T=200 N=16384")
    x_true, y = simulate(PAPER_FSV, 200, 7)
    r = smc.FSVFilter(ctx, PAPER_FSV, y, 16384, seed=3).run(graph=True, steps_per_graph=10)
    ref = ofsv.particle_filter(y, PAPER_FSV, 16384, 3)
    _compare(r, ref, 16384)
    assert np.corrcoef(r["mean"][:, 0], x_true[1:, 0])[0, 1] > 0.5


@pytest.mark.parametrize("N,T", [(131072, 25), (1 << 20, 3)])
def test_fsv_benchmark_sizes(smc, ctx, N, T):
    """The benchmark's largest sizes (the paper's N = 131072, and 2^20) with
    all steps of the run in one chained graph replay (the benchmark replays 50)."""
    announce(f"fsv N={N} T={T}")
    _, y = simulate(PAPER_FSV, T, 7)
    r = smc.FSVFilter(ctx, PAPER_FSV, y, N, seed=3).run(graph=True, steps_per_graph=50)
    _compare(r, ofsv.particle_filter(y, PAPER_FSV, N, 3), N)


def test_fsv_rejects_bad_models(smc, ctx):
    _, y = simulate(PAPER_FSV, 5, 1)
    import dataclasses
    bad_u = dataclasses.replace(PAPER_FSV, U=((1.0, 2.0, 0.0), (2.0, 1.0, 0.0), (0.0, 0.0, 1.0)))
    with pytest.raises(smc.SmcError):
        smc.FSVFilter(ctx, bad_u, y, 64, seed=1).run(graph=False)
    unsupported = FsvModel(B=((1.0, 0.0, 0.0),) * 4, psi=(0.5,) * 4, phi=(0.9,) * 3,
                           U=PAPER_FSV.U)
    with pytest.raises(smc.SmcError):
        smc.FSVFilter(ctx, unsupported, y[:, :4], 64, seed=1).run(graph=False)


@pytest.mark.parametrize("N,T,per_call,scheme", [(5000, 40, 7, "systematic"),
                                                 (5000, 40, 10, "systematic"),
                                                 (3001, 23, 2, "stratified"),
                                                 (3001, 23, 9, "multinomial"),
                                                 (64, 12, 5, "systematic")])
def test_fsv_steps_equal_single_steps(smc, ctx, N, T, per_call, scheme):
    """fsv_steps in groups of per_call steps (odd and even, a ragged last
    group; eager and graph-replayed), each propagation taking the previous
    step's resampling itself, equals single fsv_step calls bit for bit: the
    population, log-weights, log-likelihood, ESS, resample count and moments."""
    announce(f"fsv_steps N={N} T={T} per_call={per_call} {scheme}")
    _, y = simulate(PAPER_FSV, T, 13)
    runs = []
    for graph, chained in ((False, False), (False, True), (True, True)):
        f = smc.FSVFilter(ctx, PAPER_FSV, y, N, seed=21, scheme=scheme)
        f.run(graph=graph, steps_per_graph=per_call, chained=chained)
        runs.append((f.x.cpu().numpy(), f.logw.cpu().numpy(), f.stats.cpu().numpy(),
                     f.moments.cpu().numpy(), int(f.t.item())))
    base = runs[0]
    assert base[2][2] > 0                                # some steps resampled
    for r in runs[1:]:
        for a, b in zip(r[:4], base[:4]):
            assert np.array_equal(a, b)
        assert r[4] == base[4] == T + 1


def test_fsv_steps_rejects_bad_arguments(smc, ctx):
    _, y = simulate(PAPER_FSV, 6, 1)
    f = smc.FSVFilter(ctx, PAPER_FSV, y, 500, seed=2)
    f.init()
    for n_steps, x_tmp in ((0, f.x_tmp), (-1, f.x_tmp), (3, f.x)):
        with pytest.raises(smc.SmcError):
            smc.fsv_steps(ctx, PAPER_FSV, f.y, f.x, x_tmp, f.logw, f.t, n_steps, 2, 0.5,
                          f.stats, f.moments, stream=f.stream)
    f.stream.synchronize()
    assert f.t.item() == 1 and f.stats.cpu().numpy()[2] == 0.0
