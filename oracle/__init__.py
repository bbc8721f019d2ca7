"""FP64 CPU oracle for the sliding-ball reconstruction hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library (``paper_2601_00551_amd``) and never imports it.

Every function follows the definition the paper states (section 4 of
"SlingBAG Pro", arXiv 2601.00551), written plainly and in FP64:

* :func:`simulate` / :func:`vjp` -- the forward model ``Simulate`` of
  section 4.2/4.3 and its vector-Jacobian product (gradients by forward-mode
  dual numbers in ``sbp_oracle.c``);
* :func:`downsample` -- ``Downsample_{f_k}`` of section 4.3 (bin average);
* :func:`residual_loss` -- the squared L2 data-fidelity loss of section 4.2/4.3;
* :func:`filter_zero_grad` -- zero-gradient filtering, section 4.2 and
  Algorithm 1;
* :func:`adam_step` -- the optimiser (PyTorch Adam semantics; the paper names
  none, section 2.1 only says all learning rates are shared);
* :func:`softplus` / :func:`softplus_inv` -- the positivity reparameterisation
  of section 4.3;
* :func:`grow` -- the split / destroy / duplicate growth rule of section 4.1
  (thresholds are not given by the paper; parity unpinned).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

UNIFORM, GAUSS = 0, 1
OMNI, COS = 0, 1
BIN, POINT = 0, 1
PARAMS = ("x", "y", "z", "p0", "a")


@dataclasses.dataclass
class Time:
    """One level of the time grid: sample n is the bin [t0 + n*f*dt, t0 + (n+1)*f*dt)."""
    c: float = 1.5          # speed of sound, mm/us (1500 m/s, paper section 2.1)
    dt: float = 0.025       # base sample interval, us
    t0: float = 0.0         # first edge, us
    T: int = 512            # samples at this level (T_k)
    f: int = 1              # downsampling factor f_k
    profile: int = GAUSS
    directivity: int = COS
    K: float = 5.0          # GAUSS truncation, in units of a
    sampling: int = BIN


class _CTime(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("dt", ctypes.c_double), ("t0", ctypes.c_double),
                ("K", ctypes.c_double), ("T", ctypes.c_int32), ("f", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("directivity", ctypes.c_int32),
                ("sampling", ctypes.c_int32), ("pad_", ctypes.c_int32)]


_LIB_PATH = os.path.join(_HERE, "liboracle.so")


def use_library(path: str) -> None:
    """Load the C part from another build of sbp_oracle.c (e.g. the
    -march=native copy); takes effect before the first call."""
    global _LIB, _LIB_PATH
    _LIB, _LIB_PATH = None, path


def _lib():
    global _LIB
    if _LIB is None:
        path = _LIB_PATH
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built (run oracle/build.py)")
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.orc_simulate.argtypes = [ctypes.c_int64] + [P] * 5 + [ctypes.c_int32] + [P] * 6 + \
            [ctypes.POINTER(_CTime), ctypes.c_int32, P, P]
        lib.orc_simulate.restype = None
        lib.orc_vjp.argtypes = [ctypes.c_int64] + [P] * 5 + [ctypes.c_int32] + [P] * 6 + \
            [ctypes.POINTER(_CTime), P, ctypes.c_int64, P, P]
        lib.orc_vjp.restype = None
        lib.orc_num_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def num_threads() -> int:
    return int(_lib().orc_num_threads())


def set_threads(n: int) -> int:
    """Use n OpenMP threads from now on; returns the number in use."""
    return int(_lib().orc_set_threads(int(n)))


def _ctime(tm: Time) -> _CTime:
    return _CTime(float(tm.c), float(tm.dt), float(tm.t0), float(tm.K), int(tm.T), int(tm.f),
                  int(tm.profile), int(tm.directivity), int(tm.sampling), 0)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _balls64(balls):
    return [_f64(balls[k]) for k in PARAMS]


def _array64(arr):
    return [_f64(arr[k]) for k in ("qx", "qy", "qz", "nx", "ny", "nz")]


def _finite_balls(b) -> np.ndarray:
    """Per ball: every one of x, y, z, p0, a is finite."""
    ok = np.ones(b[0].shape[0], dtype=bool)
    for a in b:
        ok &= np.isfinite(a)
    return ok


def simulate(balls, array, tm: Time, det_idx=None) -> np.ndarray:
    """Simulated signals y[D][T_k] (or rows ``det_idx`` only), FP64.

    Inputs may be FP32; they are widened to FP64 exactly.  Invalid input (a
    convention of the library's interface, which the paper does not cover): if
    any ball has a non-finite parameter, every sample is NaN.
    """
    b = _balls64(balls)
    q = _array64(array)
    B = b[0].shape[0]
    D = q[0].shape[0]
    if det_idx is None:
        R, idx = D, None
    else:
        idx = np.ascontiguousarray(np.asarray(det_idx, dtype=np.int32))
        R = idx.shape[0]
    y = np.zeros((R, tm.T), dtype=np.float64)
    ct = _ctime(tm)
    if not np.all(_finite_balls(b)):
        y[:] = np.nan
        return y
    _lib().orc_simulate(B, *[_ptr(a) for a in b], D, *[_ptr(a) for a in q], ctypes.byref(ct),
                        R, None if idx is None else _ptr(idx), _ptr(y))
    return y


def vjp(balls, array, tm: Time, v, ball_idx=None) -> dict:
    """Vector-Jacobian product: for each selected ball, sum_{d,n} v[d,n] dy[d,n]/dtheta.

    Returns a dict of FP64 arrays keyed by x, y, z, p0, a.  A ball with a
    non-finite parameter gets NaN in all five (interface convention for invalid
    input, as in :func:`simulate`).
    """
    b = _balls64(balls)
    q = _array64(array)
    B = b[0].shape[0]
    D = q[0].shape[0]
    v = _f64(v)
    assert v.shape == (D, tm.T), (v.shape, D, tm.T)
    if ball_idx is None:
        J, idx = B, None
    else:
        idx = np.ascontiguousarray(np.asarray(ball_idx, dtype=np.int64))
        J = idx.shape[0]
    g = np.zeros((5, J), dtype=np.float64)
    ct = _ctime(tm)
    _lib().orc_vjp(B, *[_ptr(a) for a in b], D, *[_ptr(a) for a in q], ctypes.byref(ct), _ptr(v),
                   J, None if idx is None else _ptr(idx), _ptr(g))
    bad = ~_finite_balls(b)
    if bad.any():
        sel = np.arange(B) if idx is None else idx
        g[:, bad[sel]] = np.nan
    return {k: g[i] for i, k in enumerate(PARAMS)}


def downsample(y, f: int) -> np.ndarray:
    """Downsample_f along the last axis: mean of f consecutive samples over full
    bins, T_k = floor(T / f); a tail that does not fill a bin is dropped."""
    y = _f64(y)
    T = y.shape[-1]
    Tk = T // f
    out = np.zeros(y.shape[:-1] + (Tk,), dtype=np.float64)
    for j in range(f):
        out += y[..., j:Tk * f:f]
    return out / f


def decimate(y, f: int) -> np.ndarray:
    """Keep every f-th sample along the last axis, T_k = floor(T / f): the
    pyramid of point-sampled records (the value at t0 + n f dt is sample n f
    of the full-rate record)."""
    y = _f64(y)
    Tk = y.shape[-1] // f
    return y[..., 0:Tk * f:f].copy()


def residual_loss(y_sim, y_ref):
    """Loss L = sum (y_sim - y_ref)^2 (a sum, no 1/N) and its cotangent dL/dy = 2 e."""
    e = _f64(y_sim) - _f64(y_ref)
    return float(np.sum(e * e)), 2.0 * e


def filter_zero_grad(balls, array, tm: Time, y_ref, strict: bool = True):
    """Zero-gradient filtering (section 4.2, Algorithm 1).

    Save p0, set every p0 to 0, simulate, take L = ||y_sim - y_ref||^2, back-
    propagate to g_i = dL/dp0_i, keep balls with g_i < 0 (strict, Algorithm 1;
    g_i <= 0 when ``strict`` is False, the equations of section 4.2), restore the
    saved p0 of the kept balls.  Returns (keep mask, g, compacted balls).

    Invalid input (interface convention): a ball with a non-finite parameter
    gets g = NaN and is dropped; the others are filtered as if it were absent.
    """
    saved = _f64(balls["p0"]).copy()
    zeroed = {k: _f64(balls[k]) for k in PARAMS}
    zeroed["p0"] = np.zeros_like(saved)
    fin = _finite_balls(_balls64(balls))
    sub = {k: zeroed[k][fin] for k in PARAMS}
    y_sim = simulate(sub, array, tm)
    _, v = residual_loss(y_sim, y_ref)
    g = np.full(len(saved), np.nan)
    g[fin] = vjp(sub, array, tm, v)["p0"]
    keep = g < 0.0 if strict else g <= 0.0
    out = {k: np.asarray(balls[k])[keep] for k in PARAMS}
    out["p0"] = saved[keep]
    return keep, g, out


def adam_step(param, grad, m, v, step: int, lr: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update with PyTorch semantics (bias correction, eps outside the
    square root), in FP64.  ``step`` is the 1-based step count after this update.
    Returns (param, m, v)."""
    param, grad, m, v = (_f64(a).copy() for a in (param, grad, m, v))
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    bc1 = 1.0 - beta1 ** step
    bc2 = 1.0 - beta2 ** step
    denom = np.sqrt(v) / np.sqrt(bc2) + eps
    param = param - (lr / bc1) * m / denom
    return param, m, v


def softplus(x):
    """a = log(1 + exp(x)) (section 4.3)."""
    x = _f64(x)
    return np.log1p(np.exp(-np.abs(x))) + np.maximum(x, 0.0)


def softplus_inv(a):
    """The x with softplus(x) = a, a > 0."""
    a = _f64(a)
    return a + np.log(-np.expm1(-a))


def sigmoid(x):
    x = _f64(x)
    return 1.0 / (1.0 + np.exp(-x))


@dataclasses.dataclass
class GrowthRule:
    """Thresholds of the plain growth rule (the paper gives none; section 4.1).

    The interface passes the thresholds as float32 fields, so the rule is
    defined on their float32 values, compared with the float32 ball
    parameters: the destroy threshold is destroy_frac * max p0 rounded to
    float32, and the duplicate count floor(n * dup_frac) is exact for the
    float32 dup_frac (0.7 is 0.699999988: ten candidates give six clones).
    """
    destroy_frac: float = 0.02     # destroy if p0 < destroy_frac * max p0 (per frame)
    a_min: float = 0.02            # destroy if a < a_min (mm)
    a_split: float = 0.3           # split if a > a_split (mm); default 2 * a_init
    dup_frac: float = 0.0          # duplicate the top dup_frac of candidates by |grad r|
    dup_offset: float = 0.5        # clone offset, in units of a, against grad r


def grow(balls, grads, rule: GrowthRule, ball_off=None):
    """Plain growth rule on each frame [ball_off[f], ball_off[f+1]).

    Per frame, in this order:
      1. destroy: p0 < destroy_frac * max(p0 of the frame) or a < a_min;
      2. split every survivor with a > a_split into two children placed at
         -/+ a/2 along the axis of its largest |position gradient| (ties go to
         x, then y, then z), each with size a / 2^(1/3) and the parent's p0;
      3. duplicate: among survivors that were not split, the
         floor(dup_frac * count) with the largest |grad r|^2 (ties: lower index)
         each get a clone at r - dup_offset * a * grad r / |grad r| (clones of a
         ball with zero position gradient sit on the ball).
    Output of a frame: survivors in input order, a split ball replaced in place
    by its (-, +) children, followed by the clones in input order.  Returns
    (new balls as FP64 dict, new ball_off, born mask -- True for balls whose
    optimiser moments start at zero -- and the source index of each output ball).
    """
    n_all = len(np.asarray(balls["x"]))
    if ball_off is None:
        ball_off = [0, n_all]
    f32 = np.float32
    out = {k: [] for k in PARAMS}
    born, src = [], []
    new_off = [0]
    for fr in range(len(ball_off) - 1):
        lo, hi = int(ball_off[fr]), int(ball_off[fr + 1])
        p0 = np.asarray(balls["p0"], dtype=f32)[lo:hi]
        a = np.asarray(balls["a"], dtype=f32)[lo:hi]
        n = hi - lo
        if n == 0:
            new_off.append(new_off[-1])
            continue
        pmax = np.max(p0)
        thr_p = f32(f32(rule.destroy_frac) * pmax)
        alive = ~((p0 < thr_p) | (a < f32(rule.a_min)))
        split = alive & (a > f32(rule.a_split))
        gx = np.asarray(grads["x"], dtype=f32)[lo:hi].astype(np.float64)
        gy = np.asarray(grads["y"], dtype=f32)[lo:hi].astype(np.float64)
        gz = np.asarray(grads["z"], dtype=f32)[lo:hi].astype(np.float64)
        key = (gx * gx + gy * gy) + gz * gz
        cand = np.nonzero(alive & ~split)[0]
        k = int(np.floor(len(cand) * float(f32(rule.dup_frac))))
        dup = np.zeros(n, dtype=bool)
        if k > 0:
            order = sorted(cand.tolist(), key=lambda i: (-key[i], i))
            dup[np.array(order[:k], dtype=np.int64)] = True
        count = 0
        for i in range(n):
            if not alive[i]:
                continue
            g_abs = [abs(float(grads[ax][lo + i])) for ax in ("x", "y", "z")]
            if split[i]:
                axis = int(np.argmax(g_abs))   # first maximum: x, then y, then z
                for sgn in (-1.0, 1.0):
                    for ax_i, ax in enumerate(("x", "y", "z")):
                        pos = float(balls[ax][lo + i])
                        if ax_i == axis:
                            pos += sgn * 0.5 * float(a[i])
                        out[ax].append(pos)
                    out["p0"].append(float(p0[i]))
                    out["a"].append(float(a[i]) / 2.0 ** (1.0 / 3.0))
                    born.append(True)
                    src.append(lo + i)
                    count += 1
            else:
                for k_ in PARAMS:
                    out[k_].append(float(balls[k_][lo + i]))
                born.append(False)
                src.append(lo + i)
                count += 1
        for i in range(n):
            if not dup[i]:
                continue
            gvec = np.array([float(grads[ax][lo + i]) for ax in ("x", "y", "z")])
            norm = float(np.sqrt(key[i]))
            step = np.zeros(3) if norm == 0.0 else -rule.dup_offset * float(a[i]) * gvec / norm
            for ax_i, ax in enumerate(("x", "y", "z")):
                out[ax].append(float(balls[ax][lo + i]) + step[ax_i])
            out["p0"].append(float(p0[i]))
            out["a"].append(float(a[i]))
            born.append(True)
            src.append(lo + i)
            count += 1
        new_off.append(new_off[-1] + count)
    res = {k: np.array(v, dtype=np.float64) for k, v in out.items()}
    return res, np.array(new_off, dtype=np.int64), np.array(born, dtype=bool), np.array(src, dtype=np.int64)
