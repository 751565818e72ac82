"""Thin Python binding of the C ABI: same names, torch tensors in, no arithmetic.

Every function checks tensor placement, dtype, shape and contiguity, passes raw
device pointers and the current (or given) HIP stream to libsmcgpu, and raises
``SmcError`` on a non-zero return code. Nothing here computes any part of the
sampler.
"""

from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import Optional, Sequence

import torch

from . import _lib as L

PREC = {"fp64": L.SMC_PREC_FP64, "fp32": L.SMC_PREC_FP32, "bf16x3": L.SMC_PREC_BF16X3}
PURPOSE = {"prior": 1, "prop": 2, "acc": 3, "resamp": 4, "exch": 5, "parity": 6}
SCHEME = {"systematic": L.SMC_RESAMPLE_SYSTEMATIC, "stratified": L.SMC_RESAMPLE_STRATIFIED,
          "multinomial": L.SMC_RESAMPLE_MULTINOMIAL}


@dataclasses.dataclass(frozen=True)
class Gmm:
    """Mixture model of the C ABI's smc_gmm (known weights and covariance sigma2*I)."""
    k: int
    d: int
    sigma2: float
    log_w: Sequence[float]
    prior: str = "gauss"        # "gauss": N(prior_a, prior_b^2); "box": U[prior_a, prior_b]
    prior_a: float = 0.0
    prior_b: float = 10.0

    @staticmethod
    def equal_weights(k: int, d: int, sigma2: float, **kw) -> "Gmm":
        return Gmm(k=k, d=d, sigma2=sigma2, log_w=tuple([math.log(1.0 / k)] * k), **kw)

    @property
    def kd(self) -> int:
        return self.k * self.d

    def struct(self) -> L.SmcGmm:
        s = L.SmcGmm()
        s.k = self.k
        s.d = self.d
        s.sigma2 = float(self.sigma2)
        for i in range(L.SMC_KMAX):
            s.log_w[i] = float(self.log_w[i]) if i < self.k else float("-inf")
        s.prior = {"gauss": L.SMC_PRIOR_GAUSS, "box": L.SMC_PRIOR_BOX}[self.prior]
        s.prior_a = float(self.prior_a)
        s.prior_b = float(self.prior_b)
        return s


def _prec(p) -> int:
    return PREC[p] if isinstance(p, str) else int(p)


def _stream(stream) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor, dtype, name: str, numel: Optional[int] = None) -> ctypes.c_void_p:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _opt(t, dtype, name, numel=None):
    return None if t is None else _ptr(t, dtype, name, numel)


def _data_shape(model: Gmm, y: torch.Tensor) -> int:
    if y.dim() == 1 and model.d == 1:
        return y.shape[0]
    if y.dim() == 2 and y.shape[1] == model.d:
        return y.shape[0]
    raise ValueError(f"y must be [n] (d = 1) or [n, {model.d}]")


def _theta_shape(model: Gmm, theta: torch.Tensor) -> int:
    if theta.dim() != 2 or theta.shape[0] != model.kd:
        raise ValueError(f"theta must be [k*d = {model.kd}, N]")
    return theta.shape[1]


class Context:
    """Owns an smc_ctx (device scratch and launch choices) on one GPU."""

    def __init__(self, device: int = 0):
        self._lib = L.load()
        h = ctypes.c_void_p()
        L.check(self._lib.smc_create(ctypes.byref(h), int(device)))
        self.handle = h
        self.device = device
        self.rules: list = []          # the launch table last installed

    def reserve(self, N: int, kd: int = 8, n: int = 0) -> None:
        L.check(self._lib.smc_reserve(self.handle, int(N), int(kd), int(n)))

    def check(self, stream=None) -> None:
        L.check(self._lib.smc_check(self.handle, _stream(stream)))

    def set_slices(self, slices: int) -> None:
        L.check(self._lib.smc_set_slices(self.handle, int(slices)))

    def set_pt_single_workgroup(self, mode: int) -> None:
        """pt_iterations' single-workgroup form: 0 automatic, 1 whenever the
        population fits, -1 never."""
        L.check(self._lib.pt_set_single_workgroup(self.handle, int(mode)))

    def set_resampling(self, scheme: str) -> None:
        """Resampling scheme of later smc_step / smc_step_batched calls."""
        L.check(self._lib.smc_set_resampling(self.handle, SCHEME[scheme]))

    def set_launch_table(self, rules: Sequence[dict]) -> None:
        """Install launch rules (dicts with k, d, prec, kind, slices, n_lo, n_hi,
        N_lo, N_hi; prec is a name of PREC or "any"; kind is "call" (default)
        or "batch"); an empty list clears the table."""
        arr = (L.SmcLaunchRule * max(1, len(rules)))()
        for i, r in enumerate(rules):
            prec = r.get("prec", "any")
            kind = {"call": L.SMC_RULE_CALL, "batch": L.SMC_RULE_BATCH}[r.get("kind", "call")]
            arr[i] = L.SmcLaunchRule(int(r.get("k", 0)), int(r.get("d", 0)),
                                     -1 if prec == "any" else PREC[prec], kind, int(r["slices"]),
                                     int(r["n_lo"]), int(r["n_hi"]), int(r["N_lo"]), int(r["N_hi"]))
        L.check(self._lib.smc_set_launch_table(self.handle, arr, len(rules)))
        self.rules = [dict(r) for r in rules]

    def fp32_form_counts(self, reset: bool = False) -> dict:
        """Form counts of the FP32 single moves on this device since the last
        reset (smc_fp32_form_counts), in (observation, tile) pairs: "shifted"
        (plain shifted form), "pivot" (pivot form) and "pivot_terms" (other
        components the pivot form evaluated, summed over its pairs)."""
        v = (ctypes.c_uint64 * 3)()
        L.check(self._lib.smc_fp32_form_counts(self.handle, v, int(bool(reset))))
        return {"shifted": int(v[0]), "pivot": int(v[1]), "pivot_terms": int(v[2])}

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            self._lib.smc_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def smc_loglik(ctx: Context, model: Gmm, y, theta, prec="fp32", out=None, stream=None):
    n = _data_shape(model, y)
    N = _theta_shape(model, theta)
    if out is None:
        out = torch.empty(N, dtype=torch.float64, device=theta.device)
    L.check(ctx._lib.smc_loglik(ctx.handle, ctypes.byref(model.struct()),
                                _ptr(y, torch.float32, "y"), n,
                                _ptr(theta, torch.float64, "theta"), N, _prec(prec),
                                _ptr(out, torch.float64, "loglik", N), _stream(stream)))
    return out


def smc_prior_init(ctx: Context, model: Gmm, N: int, seed: int, out=None, stream=None):
    if out is None:
        out = torch.empty((model.kd, N), dtype=torch.float64, device="cuda")
    L.check(ctx._lib.smc_prior_init(ctx.handle, ctypes.byref(model.struct()), int(N),
                                    int(seed), _ptr(out, torch.float64, "theta", model.kd * N),
                                    _stream(stream)))
    return out


def smc_rwmh_move(ctx: Context, model: Gmm, y, theta, loglik, beta, step_sd, seed, step,
                  move=0, prec="fp32", n_accept=None, beta_vec=None, stream=None):
    n = _data_shape(model, y)
    N = _theta_shape(model, theta)
    L.check(ctx._lib.smc_rwmh_move(
        ctx.handle, ctypes.byref(model.struct()), _ptr(y, torch.float32, "y"), n,
        _ptr(theta, torch.float64, "theta"), _ptr(loglik, torch.float64, "loglik", N), N,
        _opt(beta_vec, torch.float64, "beta_vec", N), float(beta), float(step_sd), int(seed),
        int(step), int(move), _prec(prec), _opt(n_accept, torch.int64, "n_accept", 1),
        _stream(stream)))


def smc_reweight(ctx: Context, logw, loglik, dbeta, W=None, logZ=None, ess=None, stream=None):
    N = logw.numel()
    L.check(ctx._lib.smc_reweight(ctx.handle, _ptr(logw, torch.float64, "logw"),
                                  _ptr(loglik, torch.float64, "loglik", N), N, float(dbeta),
                                  _opt(W, torch.float64, "W", N),
                                  _opt(logZ, torch.float64, "logZ", 1),
                                  _opt(ess, torch.float64, "ess", 1), _stream(stream)))


def smc_ess(ctx: Context, W, ess, stream=None):
    L.check(ctx._lib.smc_ess(ctx.handle, _ptr(W, torch.float64, "W"), W.numel(),
                             _ptr(ess, torch.float64, "ess", 1), _stream(stream)))


def smc_resample_systematic(ctx: Context, W, seed, step, u_override=None, ess=None,
                            ess_threshold=0.0, idx=None, theta_in=None, theta_out=None,
                            l_in=None, l_out=None, logw=None, stream=None):
    N = W.numel()
    kd = 0
    if theta_in is not None:
        if theta_in.dim() != 2 or theta_in.shape[1] != N:
            raise ValueError("theta_in must be [kd, N]")
        kd = theta_in.shape[0]
    L.check(ctx._lib.smc_resample_systematic(
        ctx.handle, _ptr(W, torch.float64, "W"), N, int(seed), int(step),
        _opt(u_override, torch.float64, "u_override", 1), _opt(ess, torch.float64, "ess", 1),
        float(ess_threshold), _opt(idx, torch.int32, "idx", N),
        _opt(theta_in, torch.float64, "theta_in", kd * N),
        _opt(theta_out, torch.float64, "theta_out", kd * N), kd,
        _opt(l_in, torch.float64, "l_in", N), _opt(l_out, torch.float64, "l_out", N),
        _opt(logw, torch.float64, "logw", N), _stream(stream)))


def smc_resample(ctx: Context, W, scheme, seed, step, ess=None, ess_threshold=0.0, idx=None,
                 theta_in=None, theta_out=None, l_in=None, l_out=None, logw=None, stream=None):
    N = W.numel()
    kd = 0
    if theta_in is not None:
        if theta_in.dim() != 2 or theta_in.shape[1] != N:
            raise ValueError("theta_in must be [kd, N]")
        kd = theta_in.shape[0]
    L.check(ctx._lib.smc_resample(
        ctx.handle, SCHEME[scheme], _ptr(W, torch.float64, "W"), N, int(seed), int(step),
        _opt(ess, torch.float64, "ess", 1), float(ess_threshold),
        _opt(idx, torch.int32, "idx", N), _opt(theta_in, torch.float64, "theta_in", kd * N),
        _opt(theta_out, torch.float64, "theta_out", kd * N), kd,
        _opt(l_in, torch.float64, "l_in", N), _opt(l_out, torch.float64, "l_out", N),
        _opt(logw, torch.float64, "logw", N), _stream(stream)))


def pt_exchange(ctx: Context, theta, loglik, beta, parity, wrap, seed, iteration, n_swap=None,
                stream=None):
    M = loglik.numel()
    if theta.dim() != 2 or theta.shape[1] != M:
        raise ValueError("theta must be [kd, M]")
    L.check(ctx._lib.pt_exchange(ctx.handle, _ptr(theta, torch.float64, "theta"),
                                 _ptr(loglik, torch.float64, "loglik"),
                                 _ptr(beta, torch.float64, "beta", M), M, theta.shape[0],
                                 int(parity), int(bool(wrap)), int(seed), int(iteration),
                                 _opt(n_swap, torch.int32, "n_swap", 1), _stream(stream)))


def smc_step(ctx: Context, model: Gmm, y, theta_in, loglik_in, theta_out, loglik_out, logw, W,
             beta, t_dev, step_sd, n_moves, seed, ess_frac, prec, stats, n_accept=None,
             stream=None):
    n = _data_shape(model, y)
    N = _theta_shape(model, theta_in)
    L.check(ctx._lib.smc_step(
        ctx.handle, ctypes.byref(model.struct()), _ptr(y, torch.float32, "y"), n, N,
        _ptr(theta_in, torch.float64, "theta_in", model.kd * N),
        _ptr(loglik_in, torch.float64, "loglik_in", N),
        _ptr(theta_out, torch.float64, "theta_out", model.kd * N),
        _ptr(loglik_out, torch.float64, "loglik_out", N),
        _ptr(logw, torch.float64, "logw", N), _ptr(W, torch.float64, "W", N),
        _ptr(beta, torch.float64, "beta"), beta.numel() - 1, _ptr(t_dev, torch.int32, "t_dev", 1),
        float(step_sd), int(n_moves), int(seed), float(ess_frac), _prec(prec),
        _ptr(stats, torch.float64, "stats", 4), _opt(n_accept, torch.int64, "n_accept", 1),
        _stream(stream)))


def smc_steps(ctx: Context, model: Gmm, y, theta_a, loglik_a, theta_b, loglik_b, logw, W, beta,
              t_dev, n_steps, step_sd, n_moves, seed, ess_frac, prec, stats, n_accept=None,
              stream=None):
    """n_steps tempering steps alternating between the (a) and (b) populations
    (even step indices read a); see smc.h."""
    n = _data_shape(model, y)
    N = _theta_shape(model, theta_a)
    L.check(ctx._lib.smc_steps(
        ctx.handle, ctypes.byref(model.struct()), _ptr(y, torch.float32, "y"), n, N,
        _ptr(theta_a, torch.float64, "theta_a", model.kd * N),
        _ptr(loglik_a, torch.float64, "loglik_a", N),
        _ptr(theta_b, torch.float64, "theta_b", model.kd * N),
        _ptr(loglik_b, torch.float64, "loglik_b", N),
        _ptr(logw, torch.float64, "logw", N), _ptr(W, torch.float64, "W", N),
        _ptr(beta, torch.float64, "beta"), beta.numel() - 1, _ptr(t_dev, torch.int32, "t_dev", 1),
        int(n_steps), float(step_sd), int(n_moves), int(seed), float(ess_frac), _prec(prec),
        _ptr(stats, torch.float64, "stats", 4), _opt(n_accept, torch.int64, "n_accept", 1),
        _stream(stream)))


def pt_iteration(ctx: Context, model: Gmm, y, theta, loglik, beta, it_dev, step_sd, seed,
                 parity_mode=0, wrap=False, prec="fp32", n_accept=None, n_swap=None,
                 stream=None):
    n = _data_shape(model, y)
    M = _theta_shape(model, theta)
    L.check(ctx._lib.pt_iteration(
        ctx.handle, ctypes.byref(model.struct()), _ptr(y, torch.float32, "y"), n, M,
        _ptr(theta, torch.float64, "theta"), _ptr(loglik, torch.float64, "loglik", M),
        _ptr(beta, torch.float64, "beta", M), _ptr(it_dev, torch.int32, "it_dev", 1),
        float(step_sd), int(seed), int(parity_mode), int(bool(wrap)), _prec(prec),
        _opt(n_accept, torch.int64, "n_accept", 1), _opt(n_swap, torch.int32, "n_swap", 1),
        _stream(stream)))


def pt_iterations(ctx: Context, model: Gmm, y, theta, loglik, beta, it_dev, n_iters, step_sd,
                  seed, parity_mode=0, wrap=False, prec="fp32", n_accept=None, n_swap=None,
                  stream=None):
    n = _data_shape(model, y)
    M = _theta_shape(model, theta)
    L.check(ctx._lib.pt_iterations(
        ctx.handle, ctypes.byref(model.struct()), _ptr(y, torch.float32, "y"), n, M,
        _ptr(theta, torch.float64, "theta"), _ptr(loglik, torch.float64, "loglik", M),
        _ptr(beta, torch.float64, "beta", M), _ptr(it_dev, torch.int32, "it_dev", 1),
        int(n_iters), float(step_sd), int(seed), int(parity_mode), int(bool(wrap)), _prec(prec),
        _opt(n_accept, torch.int64, "n_accept", 1), _opt(n_swap, torch.int32, "n_swap", 1),
        _stream(stream)))


def pt_record(ctx: Context, theta, chain, it_dev, out, stream=None):
    """out[it - 1] = theta[:, chain] after iteration it (out: [max_iters, kd] FP64)."""
    kd, M = theta.shape
    if out.dim() != 2 or out.shape[1] != kd:
        raise ValueError("out must be [max_iters, kd]")
    L.check(ctx._lib.pt_record(ctx.handle, _ptr(theta, torch.float64, "theta"), M, kd, int(chain),
                               _ptr(it_dev, torch.int32, "it_dev", 1),
                               _ptr(out, torch.float64, "out"), out.shape[0], _stream(stream)))


def _fsv_struct(model) -> "L.SmcFsv":
    """smc_fsv from any object with B (m x k), psi (m), phi (k), U (k x k)."""
    st = L.SmcFsv()
    m, k = len(model.psi), len(model.phi)
    st.m, st.k = m, k
    for i in range(m):
        st.psi[i] = float(model.psi[i])
        for c in range(k):
            st.B[i * L.SMC_FSV_KMAX + c] = float(model.B[i][c])
    for c in range(k):
        st.phi[c] = float(model.phi[c])
        for j in range(k):
            st.U[c * L.SMC_FSV_KMAX + j] = float(model.U[c][j])
    return st


def fsv_init(ctx: Context, x, logw, stream=None):
    k, N = x.shape
    L.check(ctx._lib.fsv_init(ctx.handle, k, N, _ptr(x, torch.float64, "x"),
                              _ptr(logw, torch.float64, "logw", N), _stream(stream)))


def fsv_step(ctx: Context, model, y, x, x_tmp, logw, t_dev, seed, ess_frac, stats, moments,
             stream=None):
    """One particle-filter step of the factor stochastic-volatility model
    (C ABI fsv_step); y: [T, m] FP64 device tensor."""
    T = y.shape[0]
    k, N = x.shape
    L.check(ctx._lib.fsv_step(
        ctx.handle, ctypes.byref(_fsv_struct(model)), _ptr(y, torch.float64, "y"), T, N,
        _ptr(x, torch.float64, "x"), _ptr(x_tmp, torch.float64, "x_tmp", k * N),
        _ptr(logw, torch.float64, "logw", N), _ptr(t_dev, torch.int32, "t_dev", 1), int(seed),
        float(ess_frac), _ptr(stats, torch.float64, "stats", 4),
        _ptr(moments, torch.float64, "moments", T * 2 * k), _stream(stream)))


def fsv_steps(ctx: Context, model, y, x, x_tmp, logw, t_dev, n_steps, seed, ess_frac, stats,
              moments, stream=None):
    """n_steps particle-filter steps in one call (C ABI fsv_steps: each step's
    propagation takes the previous step's resampling itself)."""
    T = y.shape[0]
    k, N = x.shape
    L.check(ctx._lib.fsv_steps(
        ctx.handle, ctypes.byref(_fsv_struct(model)), _ptr(y, torch.float64, "y"), T, N,
        _ptr(x, torch.float64, "x"), _ptr(x_tmp, torch.float64, "x_tmp", k * N),
        _ptr(logw, torch.float64, "logw", N), _ptr(t_dev, torch.int32, "t_dev", 1),
        int(n_steps), int(seed), float(ess_frac), _ptr(stats, torch.float64, "stats", 4),
        _ptr(moments, torch.float64, "moments", T * 2 * k), _stream(stream)))


def smc_sort_data(y: torch.Tensor, stream=None) -> torch.Tensor:
    """Sort the FP32 device tensor y in place into ascending order
    (smc_sort_data) and return it."""
    L.check(L.load().smc_sort_data(_ptr(y, torch.float32, "y"), int(y.numel()), _stream(stream)))
    return y


def smc_rng_words(seed, count, block, step, purpose, move=0, out=None, stream=None):
    if out is None:
        out = torch.empty((count, 4), dtype=torch.int32, device="cuda")
    pur = PURPOSE[purpose] if isinstance(purpose, str) else int(purpose)
    L.check(L.load().smc_rng_words(int(seed), int(count), int(block), int(step), pur, int(move),
                                   _ptr(out, torch.int32, "out", 4 * count), _stream(stream)))
    return out


def smc_rng_normals(seed, count, per_index, step, purpose, move=0, out=None, stream=None):
    if out is None:
        out = torch.empty((per_index, count), dtype=torch.float64, device="cuda")
    pur = PURPOSE[purpose] if isinstance(purpose, str) else int(purpose)
    L.check(L.load().smc_rng_normals(int(seed), int(count), int(per_index), int(step), pur,
                                     int(move), _ptr(out, torch.float64, "out",
                                                     per_index * count), _stream(stream)))
    return out


class Batch:
    """An smc_batch: device descriptors and scratch of many independent runs."""

    def __init__(self, ctx: Context, runs, kd: int):
        arr = (L.SmcRunDesc * len(runs))()
        for i, (p_off, y_off, N, n, seed) in enumerate(runs):
            arr[i].p_off, arr[i].y_off, arr[i].N, arr[i].n, arr[i].seed = (
                int(p_off), int(y_off), int(N), int(n), int(seed))
        h = ctypes.c_void_p()
        L.check(ctx._lib.smc_batch_create(ctx.handle, arr, len(runs), int(kd), ctypes.byref(h)))
        self.ctx, self.handle, self.R = ctx, h, len(runs)

    def close(self):
        if self.handle.value:
            self.ctx._lib.smc_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def smc_step_batched(ctx: Context, batch: Batch, model: Gmm, y, theta, loglik, logw, W, beta,
                     t_dev, step_sd, n_moves, ess_frac, prec, run_stats, n_accept=None,
                     stream=None):
    L.check(ctx._lib.smc_step_batched(
        ctx.handle, batch.handle, ctypes.byref(model.struct()), _ptr(y, torch.float32, "y"),
        _ptr(theta, torch.float64, "theta"), _ptr(loglik, torch.float64, "loglik"),
        _ptr(logw, torch.float64, "logw"), _ptr(W, torch.float64, "W"),
        _ptr(beta, torch.float64, "beta"), beta.numel() - 1, _ptr(t_dev, torch.int32, "t_dev", 1),
        float(step_sd), int(n_moves), float(ess_frac), _prec(prec),
        _ptr(run_stats, torch.float64, "run_stats", 4 * batch.R),
        _opt(n_accept, torch.int64, "n_accept", 1), _stream(stream)))


class Graph:
    """An executable hipGraph captured from calls enqueued on ``stream``."""

    def __init__(self, ctx: Context, stream: torch.cuda.Stream):
        self.ctx = ctx
        self.stream = stream
        self.handle = ctypes.c_void_p()

    def __enter__(self):
        L.check(self.ctx._lib.smc_graph_begin(self.ctx.handle, _stream(self.stream)))
        return self

    def __exit__(self, exc_type, exc, tb):
        h = ctypes.c_void_p()
        rc = self.ctx._lib.smc_graph_end(self.ctx.handle, _stream(self.stream), ctypes.byref(h))
        if exc_type is None:
            L.check(rc)
            self.handle = h
        return False

    def launch(self):
        L.check(self.ctx._lib.smc_graph_launch(self.handle, _stream(self.stream)))

    def close(self):
        if self.handle.value:
            self.ctx._lib.smc_graph_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
