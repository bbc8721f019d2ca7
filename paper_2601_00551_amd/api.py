"""Python binding of the C-ABI (include/sbp.h), one function per entry point.

Argument marshalling only: tensors are checked for dtype / device / layout,
their device pointers and the current HIP stream are handed to libsbp.so, and
outputs are allocated with torch (PyTorch provides device memory and streams;
every step of the method runs in the library's HIP kernels).
"""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _abi
from ._abi import (A, ALL, COARSE, DIR_COS, DIR_OMNI, P0, PROFILE_GAUSS, PROFILE_UNIFORM, SAMPLING_BIN,
                   SAMPLING_POINT, X, XYZ, Y, Z,
                   check, lib)

PARAMS = ("x", "y", "z", "p0", "a")
ARRAY_KEYS = ("qx", "qy", "qz", "nx", "ny", "nz")


@dataclasses.dataclass
class Model:
    """One temporal level of the forward model (mirror of sbp_model)."""
    c: float = 1.5
    dt: float = 0.025
    t0: float = 0.0
    T: int = 2048
    f: int = 1
    profile: int = PROFILE_GAUSS
    directivity: int = DIR_COS
    gauss_K: float = 5.0
    a_softplus: int = 0
    sampling: int = SAMPLING_BIN   # SAMPLING_POINT: point-sampled variant (GAUSS only)
    # transducer response: taps [rows][L] (float32, device) of this level's
    # interval f dt, rows 1 or D (see with_response), and the zero-lag tap
    response: object = None
    response_zero: int = 0

    def struct(self) -> _abi.SbpModel:
        h = self.response
        if h is not None:
            _need(h, torch.float32, "response")
            if h.dim() != 2 or h.shape[1] < 1:
                raise ValueError("response must be [rows, L]")
            if not 0 <= int(self.response_zero) < h.shape[1]:
                raise ValueError("response_zero must be in [0, L)")
        return _abi.SbpModel(float(self.c), float(self.dt), float(self.t0), float(self.gauss_K),
                             int(self.T), int(self.f), int(self.profile), int(self.directivity),
                             int(self.a_softplus), int(self.sampling),
                             None if h is None else h.data_ptr(),
                             0 if h is None else int(h.shape[1]), int(self.response_zero),
                             0 if h is None else int(h.shape[0]), 0)

    def level(self, f: int, T_base: int) -> "Model":
        """The level with downsampling factor f of a record of T_base samples
        (without a response: its taps depend on the level's interval)."""
        if self.response is not None:
            raise ValueError("a model with a response: attach each level's taps with with_response")
        return dataclasses.replace(self, f=int(f), T=int(T_base) // int(f))


@dataclasses.dataclass
class GrowthRule:
    destroy_frac: float = 0.02
    a_min: float = 0.02
    a_split: float = 0.3
    dup_frac: float = 0.0
    dup_offset: float = 0.5

    def struct(self) -> _abi.SbpGrowthRule:
        return _abi.SbpGrowthRule(self.destroy_frac, self.a_min, self.a_split, self.dup_frac,
                                  self.dup_offset, 0)


@dataclasses.dataclass
class AdamParams:
    lr: tuple = (0.005, 0.005, 0.005, 0.02, 0.002)   # x, y, z, p0, a
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    step: int = 1
    mask: int = ALL

    def struct(self) -> _abi.SbpAdamParams:
        return _abi.SbpAdamParams((ctypes.c_float * 5)(*self.lr), self.beta1, self.beta2,
                                  self.eps, int(self.step), int(self.mask))


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t, dtype=torch.float32, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} CUDA tensor")
    return t


def _at_least(t, n, name):
    """The kernels index device buffers by the sizes passed beside them: a
    buffer shorter than that is a host-side error here, not a GPU fault."""
    if t is not None and t.numel() < n:
        raise ValueError(f"{name} holds {t.numel()} elements, the call needs {n}")
    return t


def _exactly(t, n, name):
    if t is not None and t.numel() != n:
        raise ValueError(f"{name} holds {t.numel()} elements, the call needs exactly {n}")
    return t


def _check_balls(b, n, what="balls"):
    for k in PARAMS:
        if b is not None and b.get(k) is not None:
            _at_least(b[k], n, f"{what}[{k!r}]")


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def array_struct(arr, dtype=torch.float32) -> _abi.SbpArray:
    ts = [_need(arr[k], dtype, k) for k in ARRAY_KEYS]
    for k, t in zip(ARRAY_KEYS, ts):
        _exactly(t, ts[0].numel(), f"array[{k!r}]")
    return _abi.SbpArray(*[t.data_ptr() for t in ts], int(ts[0].numel()), 0)


def balls_struct(b, dtype=torch.float32) -> _abi.SbpBalls:
    if b is None:
        return _abi.SbpBalls()
    return _abi.SbpBalls(*[(_need(b[k], dtype, k).data_ptr() if b.get(k) is not None else None)
                           for k in PARAMS])


def default_off(balls, device):
    n = balls["x"].numel()
    return torch.tensor([0, n], dtype=torch.int64, device=device)


class Context:
    """A library context on one device (sbp_ctx)."""

    def __init__(self, device: int = 0):
        self.ptr = ctypes.c_void_p()
        self.device = int(device)
        check(lib().sbp_ctx_create(ctypes.byref(self.ptr), self.device))

    def close(self):
        if self.ptr:
            check(lib().sbp_ctx_destroy(self.ptr))
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            if self.ptr:
                lib().sbp_ctx_destroy(self.ptr)
        except Exception:
            pass

    @property
    def num_cus(self) -> int:
        n = ctypes.c_int32()
        check(lib().sbp_ctx_num_cus(self.ptr, ctypes.byref(n)))
        return n.value

    @property
    def tuning(self) -> dict:
        t = _abi.SbpTuning()
        check(lib().sbp_ctx_get_tuning(self.ptr, ctypes.byref(t)))
        return {n: getattr(t, n) for n, _ in _abi.SbpTuning._fields_}

    @tuning.setter
    def tuning(self, d: dict):
        cur = self.tuning
        cur.update(d)
        t = _abi.SbpTuning(**cur)
        check(lib().sbp_ctx_set_tuning(self.ptr, ctypes.byref(t)))


_DEFAULT_CTX = {}


def context(device: int = 0) -> Context:
    """A process-wide default context per device."""
    if device not in _DEFAULT_CTX:
        _DEFAULT_CTX[device] = Context(device)
    return _DEFAULT_CTX[device]


# ---------------------------------------------------------------- calls ----

def simulate_signals(ctx, arr, balls, model: Model, ball_off=None, y=None, accumulate=False,
                     B_cap=None, stream=None, dtype=torch.float32, noalloc=False):
    """sbp_simulate_signals (sbp_simulate_signals_noalloc with noalloc=True,
    FP32 only): returns y [F, D, T]."""
    dev = balls["x"].device
    off = default_off(balls, dev) if ball_off is None else _need(ball_off, torch.int64, "ball_off")
    F = off.numel() - 1
    D = arr["qx"].numel()
    if y is None:
        y = torch.empty((F, D, model.T), dtype=dtype, device=dev)
    _exactly(_need(y, dtype, "y"), F * D * model.T, "y")
    cap = balls["x"].numel() if B_cap is None else int(B_cap)
    _check_balls(balls, cap)
    _at_least(off, 1, "ball_off")
    if noalloc and dtype != torch.float32:
        raise ValueError("the allocation-free forward is FP32 only")
    fn = lib().sbp_simulate_signals if dtype == torch.float32 else lib().sbp_simulate_signals_f64
    if noalloc:
        fn = lib().sbp_simulate_signals_noalloc
    check(fn(ctx.ptr, ctypes.byref(array_struct(arr, dtype)), ctypes.byref(balls_struct(balls, dtype)),
             _p(off), F, cap, ctypes.byref(model.struct()), _p(y), int(bool(accumulate)), _stream(stream)))
    return y


def adjoint_gradients(ctx, arr, balls, model: Model, v, mask=ALL, ball_off=None, grad=None,
                      B_cap=None, stream=None, dtype=torch.float32):
    """sbp_adjoint_gradients: returns {param: dL/dparam} for the parameters in mask."""
    dev = balls["x"].device
    off = default_off(balls, dev) if ball_off is None else _need(ball_off, torch.int64, "ball_off")
    F = off.numel() - 1
    n = balls["x"].numel()
    if grad is None:
        grad = {k: (torch.empty(n, dtype=dtype, device=dev) if mask & (1 << i) else None)
                for i, k in enumerate(PARAMS)}
    _need(v, dtype, "v")
    cap = n if B_cap is None else int(B_cap)
    _exactly(v, F * arr["qx"].numel() * model.T, "v")
    _check_balls(balls, cap)
    _check_balls({k: grad.get(k) for k in PARAMS if mask & (1 << PARAMS.index(k))}, cap, "grad")
    fn = lib().sbp_adjoint_gradients if dtype == torch.float32 else lib().sbp_adjoint_gradients_f64
    check(fn(ctx.ptr, ctypes.byref(array_struct(arr, dtype)), ctypes.byref(balls_struct(balls, dtype)),
             _p(off), F, cap, ctypes.byref(model.struct()), _p(v), int(mask),
             ctypes.byref(balls_struct(grad, dtype)), _stream(stream)))
    return grad


# ---------------------------------------------------- transducer response --

def response_length(fc: float, bw: float, dt_k: float, n_sigma: float = 5.0):
    """sbp_response_length: (L, zero) covering +-n_sigma envelope widths of
    the response of centre fc (MHz) and fractional bandwidth bw."""
    L, zero = _abi.I32(), _abi.I32()
    check(lib().sbp_response_length(float(fc), float(bw), float(dt_k), float(n_sigma),
                                    ctypes.byref(L), ctypes.byref(zero)))
    return int(L.value), int(zero.value)


def response_taps(ctx, fc, bw, dt_k: float, L: int, zero: int, out=None, stream=None):
    """sbp_response_taps: taps [rows, L] of the responses fc[rows] (MHz),
    bw[rows] (device float32)."""
    _need(fc, torch.float32, "fc")
    _need(bw, torch.float32, "bw")
    rows = fc.numel()
    _exactly(bw, rows, "bw")
    if out is None:
        out = torch.empty((rows, int(L)), dtype=torch.float32, device=fc.device)
    _exactly(_need(out, torch.float32, "out"), rows * int(L), "out")
    check(lib().sbp_response_taps(ctx.ptr, _p(fc), _p(bw), rows, float(dt_k), int(L), int(zero),
                                  _p(out), _stream(stream)))
    return out


def response_apply(ctx, h, zero: int, y, adjoint=False, out=None, accumulate=False, stream=None):
    """sbp_response_apply on y [..., D, T] with taps h [rows, L] (rows 1 or D):
    the convolution (adjoint=False) or the correlation."""
    _need(h, torch.float32, "h")
    _need(y, torch.float32, "y")
    if h.dim() != 2 or y.dim() < 2:
        raise ValueError("h must be [rows, L] and y [..., D, T]")
    D, T = y.shape[-2], y.shape[-1]
    R = y.numel() // T
    if out is None:
        out = torch.empty_like(y)
    _exactly(_need(out, torch.float32, "out"), y.numel(), "out")
    check(lib().sbp_response_apply(ctx.ptr, _p(h), int(h.shape[0]), int(h.shape[1]), int(zero), _p(y),
                                   R, D, T, int(bool(adjoint)), int(bool(accumulate)), _p(out),
                                   _stream(stream)))
    return out


def with_response(ctx, model: Model, fc, bw, n_sigma: float = 5.0) -> Model:
    """model with the taps of the responses (fc, bw: device float32, one entry
    or one per transducer) at its interval f dt, long enough for the widest."""
    i = int(torch.argmin(fc * bw).item())      # the widest envelope sets the length
    L, zero = response_length(float(fc[i].item()), float(bw[i].item()), model.f * model.dt, n_sigma)
    h = response_taps(ctx, fc, bw, model.f * model.dt, L, zero)
    return dataclasses.replace(model, response=h, response_zero=zero)


def simulate_signals_f64(ctx, arr, balls, model, **kw):
    return simulate_signals(ctx, arr, balls, model, dtype=torch.float64, **kw)


def adjoint_gradients_f64(ctx, arr, balls, model, v, **kw):
    return adjoint_gradients(ctx, arr, balls, model, v, dtype=torch.float64, **kw)


def residual_loss(ctx, y_sim, y_ref, v_out=None, loss=None, stream=None):
    """sbp_residual_loss over [F, D, T]: returns loss [F] (float64, device)."""
    _need(y_sim, name="y_sim")
    _need(y_ref, name="y_ref")
    F = y_sim.shape[0]
    n = y_sim[0].numel()
    if loss is None:
        loss = torch.empty(F, dtype=torch.float64, device=y_sim.device)
    _exactly(y_ref, y_sim.numel(), "y_ref")
    _exactly(v_out, y_sim.numel(), "v_out")
    _at_least(loss, F, "loss")
    check(lib().sbp_residual_loss(ctx.ptr, _p(y_sim), _p(y_ref), n, F, _p(_need(v_out, name="v_out")),
                                  _p(_need(loss, torch.float64, "loss")), _stream(stream)))
    return loss


def downsample(ctx, y, f: int, out=None, stream=None):
    """sbp_downsample along the last axis."""
    _need(y, name="y")
    T = y.shape[-1]
    R = y.numel() // T
    if f < 1:
        raise ValueError("f must be >= 1")
    if out is None:
        out = torch.empty(y.shape[:-1] + (T // f,), dtype=torch.float32, device=y.device)
    _exactly(_need(out, name="out"), R * (T // f), "out")
    check(lib().sbp_downsample(ctx.ptr, _p(y), R, T, int(f), _p(_need(out, name="out")), _stream(stream)))
    return out


def decimate(ctx, y, f: int, out=None, stream=None):
    """sbp_decimate along the last axis (keeps every f-th sample)."""
    _need(y, name="y")
    T = y.shape[-1]
    R = y.numel() // T
    if f < 1:
        raise ValueError("f must be >= 1")
    if out is None:
        out = torch.empty(y.shape[:-1] + (T // f,), dtype=torch.float32, device=y.device)
    _exactly(_need(out, name="out"), R * (T // f), "out")
    check(lib().sbp_decimate(ctx.ptr, _p(y), R, T, int(f), _p(_need(out, name="out")), _stream(stream)))
    return out


def filter_zero_grad(ctx, arr, balls, model: Model, y_ref, ball_off=None, strict=True,
                     moments=None, out=None, off_out=None, g_out=None, B_cap=None, stream=None,
                     moments_out=None):
    """sbp_filter_zero_grad.  Returns (kept balls, off_out, g, out moments or None).

    The kept balls sit in the first off_out[F] entries of the returned arrays
    (which have the input's capacity)."""
    dev = balls["x"].device
    off = default_off(balls, dev) if ball_off is None else _need(ball_off, torch.int64, "ball_off")
    F = off.numel() - 1
    n = balls["x"].numel()
    cap = n if B_cap is None else int(B_cap)
    if out is None:
        out = {k: torch.empty(n, dtype=torch.float32, device=dev) for k in PARAMS}
    if off_out is None:
        off_out = torch.empty(F + 1, dtype=torch.int64, device=dev)
    if g_out is None:
        g_out = torch.empty(n, dtype=torch.float32, device=dev)
    m_in = v_in = m_out = v_out = None
    if moments is not None:
        m_in, v_in = moments
        if moments_out is not None:
            m_out, v_out = moments_out
        else:
            m_out = {k: torch.empty_like(m_in[k]) for k in PARAMS}
            v_out = {k: torch.empty_like(v_in[k]) for k in PARAMS}
    _check_balls(balls, cap)
    _check_balls(out, cap, "out")
    for name, b in (("moments[0]", m_in), ("moments[1]", v_in), ("moments_out[0]", m_out),
                    ("moments_out[1]", v_out)):
        _check_balls(b, cap, name)
    _at_least(off_out, F + 1, "off_out")
    _at_least(g_out, cap, "g_out")
    _exactly(y_ref, F * arr["qx"].numel() * model.T, "y_ref")
    ref = lambda b: None if b is None else ctypes.byref(balls_struct(b))
    check(lib().sbp_filter_zero_grad(
        ctx.ptr, ctypes.byref(array_struct(arr)), ctypes.byref(balls_struct(balls)), _p(off), F, cap,
        ctypes.byref(model.struct()), _p(_need(y_ref, name="y_ref")), int(bool(strict)),
        ctypes.byref(balls_struct(out)), _p(off_out), _p(g_out), ref(m_in), ref(v_in), ref(m_out),
        ref(v_out), _stream(stream)))
    return out, off_out, g_out, (None if moments is None else (m_out, v_out))


class State:
    """Parameters, gradient workspace and Adam moments of one (batched)
    reconstruction, at capacity B_cap; frame f owns [ball_off[f], ball_off[f+1])."""

    def __init__(self, balls, ball_off=None, capacity=None, device="cuda"):
        n = int(len(balls["x"]))
        cap = max(n, int(capacity or n))
        self.B_cap = cap
        self.balls = {}
        for k in PARAMS:
            t = torch.zeros(cap, dtype=torch.float32, device=device)
            t[:n] = torch.as_tensor(balls[k], dtype=torch.float32, device=device)
            self.balls[k] = t
        self.grad = {k: torch.zeros(cap, dtype=torch.float32, device=device) for k in PARAMS}
        self.m = {k: torch.zeros(cap, dtype=torch.float32, device=device) for k in PARAMS}
        self.v = {k: torch.zeros(cap, dtype=torch.float32, device=device) for k in PARAMS}
        if ball_off is None:
            ball_off = [0, n]
        self.ball_off = torch.as_tensor(ball_off, dtype=torch.int64, device=device).contiguous()
        self.F = self.ball_off.numel() - 1

    def struct(self) -> _abi.SbpState:
        return _abi.SbpState(balls_struct(self.balls), balls_struct(self.grad), balls_struct(self.m),
                             balls_struct(self.v), self.ball_off.data_ptr(), self.F, 0, self.B_cap)

    def count(self) -> int:
        return int(self.ball_off[-1].item())

    def host(self):
        n = self.count()
        return {k: self.balls[k][:n].detach().cpu().numpy() for k in PARAMS}


def adam_update(ctx, state: State, params: AdamParams, step_dev=None, stream=None):
    check(lib().sbp_adam_update(ctx.ptr, ctypes.byref(state.struct()), ctypes.byref(params.struct()),
                                _p(step_dev), _stream(stream)))


def step(ctx, arr, state: State, model: Model, y_ref, y_work, params: AdamParams, loss=None,
         stream=None):
    """sbp_step: one iteration (simulate, residual+loss, adjoint, Adam).  Returns loss [F]."""
    if loss is None:
        loss = torch.empty(state.F, dtype=torch.float64, device=y_ref.device)
    n = state.F * arr["qx"].numel() * model.T
    _exactly(y_ref, n, "y_ref")
    _at_least(y_work, n, "y_work")
    _at_least(loss, state.F, "loss")
    check(lib().sbp_step(ctx.ptr, ctypes.byref(array_struct(arr)), ctypes.byref(state.struct()),
                         ctypes.byref(model.struct()), _p(_need(y_ref, name="y_ref")),
                         _p(_need(y_work, name="y_work")), ctypes.byref(params.struct()),
                         _p(_need(loss, torch.float64, "loss")), _stream(stream)))
    return loss


class StepGraph:
    """sbp_step_graph_create: `iters` iterations captured in one HIP graph."""

    def __init__(self, ctx, arr, state: State, model: Model, y_ref, y_work, params: AdamParams,
                 iters: int, step0: int = 1, stream=None):
        dev = y_ref.device
        n = state.F * arr["qx"].numel() * model.T
        _exactly(_need(y_ref, name="y_ref"), n, "y_ref")
        _at_least(_need(y_work, name="y_work"), n, "y_work")
        self.step_dev = torch.tensor([int(step0)], dtype=torch.int32, device=dev)
        self.loss = torch.zeros(iters * state.F, dtype=torch.float64, device=dev)
        self.iters = iters
        self._keep = (arr, state, y_ref, y_work)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        self.ptr = ctypes.c_void_p()
        # the capture must be on a non-default stream
        self.stream.wait_stream(torch.cuda.current_stream(dev))
        check(lib().sbp_step_graph_create(
            ctx.ptr, ctypes.byref(array_struct(arr)), ctypes.byref(state.struct()),
            ctypes.byref(model.struct()), _p(y_ref), _p(y_work), ctypes.byref(params.struct()),
            _p(self.step_dev), _p(self.loss), int(iters), ctypes.byref(self.ptr),
            ctypes.c_void_p(self.stream.cuda_stream)))

    def launch(self, stream=None):
        s = stream if stream is not None else self.stream
        check(lib().sbp_graph_launch(self.ptr, ctypes.c_void_p(s.cuda_stream)))

    def close(self):
        if self.ptr:
            check(lib().sbp_graph_destroy(self.ptr))
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            if self.ptr:
                lib().sbp_graph_destroy(self.ptr)
        except Exception:
            pass


def softplus_reparam(ctx, state: State, to_softplus: bool, stream=None):
    """sbp_softplus_reparam: a <-> a~ in place (a = softplus(a~)); resets a's moments."""
    check(lib().sbp_softplus_reparam(ctx.ptr, ctypes.byref(state.struct()), int(bool(to_softplus)),
                                     _stream(stream)))


def grow(ctx, state: State, rule: GrowthRule, capacity=None, stream=None):
    """sbp_grow: returns (new State, total count)."""
    cap = int(capacity or state.B_cap)
    dev = state.ball_off.device
    out = State({k: torch.zeros(0) for k in PARAMS}, ball_off=[0] * (state.F + 1), capacity=cap,
                device=dev)
    cnt = ctypes.c_int64()
    check(lib().sbp_grow(ctx.ptr, ctypes.byref(state.struct()), ctypes.byref(rule.struct()),
                         ctypes.byref(out.struct()), ctypes.byref(cnt), _stream(stream)))
    return out, cnt.value
