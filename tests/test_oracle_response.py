"""Pins of the transducer-response oracle (oracle/response.py) against facts
fixed outside it: the impulse response itself, numpy's convolution, the
adjoint identity, and the spectrum the paper's figures fix (section 2.2:
2.02 MHz centre frequency, 54 % bandwidth)."""
import math

import numpy as np
import pytest

from oracle import response as R

FC, BW = 2.02, 0.54


def _dtft(h, dt, f, zero):
    """Gain of the taps at frequency f (MHz), the taps taken as samples at
    lags (j - zero) dt."""
    t = (np.arange(h.shape[-1]) - zero) * dt
    return abs(np.sum(h * np.exp(-2j * math.pi * f * t)))


def test_impulse_gives_the_taps_back():
    dt = 0.025
    L, zero = R.taps_length(FC, BW, dt)
    h = R.gauss_taps(FC, BW, dt, L, zero)[0]
    T, n0 = 400, 150
    y = np.zeros(T)
    y[n0] = 1.0
    out = R.convolve(h, y, zero)
    want = np.zeros(T)
    for j in range(L):                   # an impulse at n0 shows tap j at n0 - zero + j
        n = n0 - zero + j
        if 0 <= n < T:
            want[n] = h[j]
    assert np.array_equal(out, want)


@pytest.mark.parametrize("L,zero", [(1, 0), (5, 0), (5, 4), (9, 3), (31, 15)])
def test_matches_numpy_convolve(L, zero):
    rng = np.random.default_rng(L * 10 + zero)
    h = rng.normal(size=L)
    y = rng.normal(size=(3, 200))
    out = R.convolve(h, y, zero)
    for r in range(3):
        full = np.convolve(y[r], h)        # full[m] = sum_j h[j] y[m - j]
        np.testing.assert_allclose(out[r], full[zero:zero + 200], rtol=0, atol=1e-12)


@pytest.mark.parametrize("L,zero,T", [(7, 3, 50), (31, 0, 40), (139, 69, 100), (139, 69, 30)])
def test_correlate_is_the_adjoint(L, zero, T):
    rng = np.random.default_rng(T + L)
    h = rng.normal(size=(4, L))
    y = rng.normal(size=(2, 4, T))
    v = rng.normal(size=(2, 4, T))
    lhs = np.sum(R.convolve(h, y, zero, D=4) * v)
    rhs = np.sum(y * R.correlate(h, v, zero, D=4))
    assert abs(lhs - rhs) <= 1e-12 * (np.sum(np.abs(y)) * np.sum(np.abs(v)) * np.abs(h).max())


@pytest.mark.parametrize("dt", [0.025, 0.05, 0.1])
def test_spectrum_has_unit_gain_at_fc_and_half_at_the_band_edges(dt):
    """Section 2.2's figures: gain 1 at 2.02 MHz and -6 dB (one half) at
    fc (1 +- 0.54 / 2), at every level's sample interval."""
    L, zero = R.taps_length(FC, BW, dt, n_sigma=6.0)
    h = R.gauss_taps(FC, BW, dt, L, zero)[0]
    assert _dtft(h, dt, FC, zero) == pytest.approx(1.0, abs=1e-6)
    for f in (FC * (1 - BW / 2), FC * (1 + BW / 2)):
        assert _dtft(h, dt, f, zero) == pytest.approx(0.5, abs=1e-6)
    # the gain peaks at fc
    fs = np.linspace(0.5, 4.0, 351)
    g = [_dtft(h, dt, f, zero) for f in fs]
    assert abs(fs[int(np.argmax(g))] - FC) <= 0.01


def test_per_transducer_rows_are_used_by_transducer():
    rng = np.random.default_rng(5)
    D, T, L, zero = 3, 60, 9, 4
    fc = FC * (1 + 0.05 * rng.normal(size=D))
    bw = BW * (1 + 0.05 * rng.normal(size=D))
    h = R.gauss_taps(fc, bw, 0.05, L, zero)
    y = rng.normal(size=(2, D, T))
    out = R.convolve(h, y, zero, D=D)
    for f in range(2):
        for d in range(D):
            full = np.convolve(y[f, d], h[d])
            np.testing.assert_allclose(out[f, d], full[zero:zero + T], atol=1e-12)


def test_taps_length_covers_the_envelope():
    dt = 0.025
    L, zero = R.taps_length(FC, BW, dt, n_sigma=5.0)
    assert L == 2 * zero + 1
    h = R.gauss_taps(FC, BW, dt, L, zero)[0]
    s_t = 1.0 / (2 * math.pi * BW * FC / (2 * math.sqrt(2 * math.log(2))))
    # the outermost taps sit beyond 5 envelope widths, the next ones inside
    assert zero * dt >= 5 * s_t > (zero - 1) * dt
    assert np.abs(h[[0, -1]]).max() <= math.exp(-12.5) * np.abs(h).max()
