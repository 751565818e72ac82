"""The resampling entry point that allocates nothing, smc_resample_noalloc,
called through the C ABI and checked against smc_resample (the context-scratch
entry point with the same kernels): two calls in a row, the second with fewer
particles, for every scheme; indices, gathered parameters and log-likelihoods
and the reset log-weights must be bit-identical, and both must equal the
oracle's indices. Sizes above the array's maximum are refused before any
work is enqueued."""

import ctypes

import numpy as np
import pytest
import torch

from gpu_common import announce
from oracle import smc as osmc
from workloads import lognormal_logw

pytestmark = pytest.mark.gpu


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("scheme", ["systematic", "stratified", "multinomial"])
def test_noalloc_resample_matches_context_entry_point(scheme):
    import paper_0905_2441_amd as smc
    from paper_0905_2441_amd import _lib as L
    from paper_0905_2441_amd.api import SCHEME
    lib = L.load()
    torch.cuda.set_device(0)
    ctx = smc.Context(0)
    stream = torch.cuda.current_stream()
    kd = 4
    rng = np.random.default_rng(7)
    for call, N in enumerate(((1 << 20) - 3, 70001)):
        announce(f"noalloc resample {scheme} call {call} N={N}")
        W = osmc.normalise(lognormal_logw(N, seed=call + 11))
        theta = rng.normal(size=(kd, N))
        l = rng.normal(size=N)
        Wd = torch.as_tensor(W).cuda()
        th_in = torch.as_tensor(theta).cuda()
        l_in = torch.as_tensor(l).cuda()
        outs = {}
        for which in ("context", "noalloc"):
            idx = torch.full((N,), -1, dtype=torch.int32, device="cuda")
            th_out = torch.zeros((kd, N), dtype=torch.float64, device="cuda")
            l_out = torch.zeros(N, dtype=torch.float64, device="cuda")
            logw = torch.ones(N, dtype=torch.float64, device="cuda")
            if which == "context":
                smc.smc_resample(ctx, Wd, scheme, 31, 5 + call, idx=idx, theta_in=th_in,
                                 theta_out=th_out, l_in=l_in, l_out=l_out, logw=logw)
            else:
                rc = lib.smc_resample_noalloc(SCHEME[scheme], _p(Wd), N, 31, 5 + call, None, 0.0,
                                              _p(idx), _p(th_in), _p(th_out), kd, _p(l_in),
                                              _p(l_out), _p(logw),
                                              ctypes.c_void_p(stream.cuda_stream))
                assert rc == L.SMC_OK, lib.smc_last_error()
            torch.cuda.synchronize()
            outs[which] = [t.cpu().numpy() for t in (idx, th_out, l_out, logw)]
        for a, b in zip(outs["context"], outs["noalloc"]):
            assert np.array_equal(a, b)
        ref = osmc.resample_indices(W, scheme, 31, 5 + call)
        assert np.array_equal(outs["noalloc"][0], ref)
        assert np.array_equal(outs["noalloc"][1], theta[:, ref])
        assert np.all(outs["noalloc"][3] == 0.0)
    # an ESS test that does not fire: identity and copies, logw untouched
    N = 5000
    W = np.full(N, 1.0 / N)
    ess = torch.full((1,), float(N), dtype=torch.float64, device="cuda")
    idx = torch.full((N,), -1, dtype=torch.int32, device="cuda")
    logw = torch.ones(N, dtype=torch.float64, device="cuda")
    rc = lib.smc_resample_noalloc(SCHEME[scheme], _p(torch.as_tensor(W).cuda()), N, 3, 1, _p(ess),
                                  0.5 * N, _p(idx), None, None, 0, None, None, _p(logw),
                                  ctypes.c_void_p(stream.cuda_stream))
    assert rc == L.SMC_OK
    torch.cuda.synchronize()
    assert np.array_equal(idx.cpu().numpy(), np.arange(N))
    assert np.all(logw.cpu().numpy() == 1.0)
    # above the maximum: refused, nothing enqueued
    big = (1 << 20) + 1
    rc = lib.smc_resample_noalloc(SCHEME[scheme], _p(torch.zeros(1, dtype=torch.float64,
                                                                 device="cuda")), big, 3, 1,
                                  None, 0.0, None, None, None, 0, None, None, None, None)
    assert rc == L.SMC_ERR_INVALID_ARG
    assert b"maximum" in lib.smc_last_error()
    ctx.close()
