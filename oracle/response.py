"""Transducer impulse response: FP64 oracle.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``, never by the HIP library's package.

Section 2.2 reports that the in vivo array's elements have a mean centre
frequency of 2.02 MHz and a bandwidth of 54 %; the forward model of sections
4.2 and 4.3 leaves the transducer's own response out.  Adding it makes the
modelled record the simulated pressure record convolved in time with the
element's impulse response.  Readings taken here (the paper gives no formula):

* the response is a Gaussian-envelope cosine,
  h(t) = A exp(-t^2 / (2 s_t^2)) cos(2 pi fc t), whose amplitude spectrum is
  a Gaussian centred on fc;
* "bandwidth" is the full width of that amplitude spectrum at half its peak
  (-6 dB), as a fraction of fc: s_f = bw fc / (2 sqrt(2 ln 2)), and
  s_t = 1 / (2 pi s_f);
* A makes the gain at fc one: A = 2 / (s_t sqrt(2 pi)) (the mirror lobe at
  -fc adds exp(-2 (fc / s_f)^2) to that gain, below 1e-16 at 54 %);
* at a level with sample interval dt_k the continuous convolution integral is
  replaced by the sum over taps h_j = dt_k h((j - zero) dt_k), j = 0..L-1,
  applied to that level's record with zeros outside [0, T).

Rows of signals are transducer records (frames back to back, D rows each);
row r uses tap row (r mod D) when there is one response per transducer, else
the single shared row.
"""
from __future__ import annotations

import math

import numpy as np


def gauss_taps(fc, bw, dt_k: float, L: int, zero: int) -> np.ndarray:
    """Taps [rows][L] of the Gaussian-envelope response sampled at dt_k.

    fc (MHz) and bw (fraction) are scalars or arrays of one entry per row;
    tap j sits at lag (j - zero) dt_k (us)."""
    fc = np.atleast_1d(np.asarray(fc, dtype=np.float64))
    bw = np.atleast_1d(np.asarray(bw, dtype=np.float64))
    if fc.shape != bw.shape:
        raise ValueError("fc and bw need one entry per row")
    s_f = bw * fc / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    s_t = 1.0 / (2.0 * math.pi * s_f)
    amp = 2.0 / (s_t * math.sqrt(2.0 * math.pi))
    t = (np.arange(L, dtype=np.float64) - zero) * dt_k
    env = np.exp(-(t[None, :] ** 2) / (2.0 * s_t[:, None] ** 2))
    return dt_k * amp[:, None] * env * np.cos(2.0 * math.pi * fc[:, None] * t[None, :])


def _rows(h, n_rows: int, D: int) -> np.ndarray:
    h = np.asarray(h, dtype=np.float64)
    if h.ndim == 1:
        h = h[None]
    if h.shape[0] == 1:
        return np.repeat(h, n_rows, axis=0)
    if h.shape[0] != D or n_rows % D:
        raise ValueError("tap rows must be 1 or D, and the record rows a multiple of D")
    return np.tile(h, (n_rows // D, 1))


def convolve(h, y, zero: int, D: int | None = None) -> np.ndarray:
    """out[r][n] = sum_j h[row(r)][j] y[r][n + zero - j], zeros outside the record.

    y is [..., T]; its leading axes flatten to rows (D per frame)."""
    y = np.asarray(y, dtype=np.float64)
    T = y.shape[-1]
    Y = y.reshape(-1, T)
    H = _rows(h, Y.shape[0], D or Y.shape[0])
    out = np.zeros_like(Y)
    for j in range(H.shape[1]):
        s = zero - j                      # out[n] takes y[n + s]
        lo, hi = max(0, -s), min(T, T - s)
        if lo < hi:
            out[:, lo:hi] += H[:, j:j + 1] * Y[:, lo + s:hi + s]
    return out.reshape(y.shape)


def correlate(h, v, zero: int, D: int | None = None) -> np.ndarray:
    """The adjoint of :func:`convolve`:
    out[r][n] = sum_j h[row(r)][j] v[r][n - zero + j], zeros outside the record."""
    v = np.asarray(v, dtype=np.float64)
    T = v.shape[-1]
    V = v.reshape(-1, T)
    H = _rows(h, V.shape[0], D or V.shape[0])
    out = np.zeros_like(V)
    for j in range(H.shape[1]):
        s = j - zero                      # out[n] takes v[n + s]
        lo, hi = max(0, -s), min(T, T - s)
        if lo < hi:
            out[:, lo:hi] += H[:, j:j + 1] * V[:, lo + s:hi + s]
    return out.reshape(v.shape)


def taps_length(fc_min: float, bw_min: float, dt_k: float, n_sigma: float = 5.0) -> tuple:
    """(L, zero) for taps covering +-n_sigma envelope widths of the widest
    response (the one of least fc * bw)."""
    s_t = 1.0 / (2.0 * math.pi * bw_min * fc_min / (2.0 * math.sqrt(2.0 * math.log(2.0))))
    half = int(math.ceil(n_sigma * s_t / dt_k))
    return 2 * half + 1, half
