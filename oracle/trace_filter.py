"""FP64 CPU oracle for the trace pre-filter (the rho filter of Kirchhoff
migration), applied to every trace before migration, and its transpose.

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's CPU
baseline, never by the GPU library or its binding.

The paper applies no filter to the data before the sum of Eq. (1); a
production Kirchhoff migration pre-filters the traces so that the summation
over the acquisition surface returns a zero-phase wavelet.  The filter is a
finite impulse response given as taps h[0..K-1] with h[c] at zero lag:
    forward  y[n] = sum_k h[k] x[n + c - k]   (x = 0 outside [0, N)),
    adjoint  x[m] = sum_k h[k] y[m - c + k]   (y = 0 outside [0, N)),
so <forward(x), y> = <x, adjoint(y)>.

Parity status: pinned by the CPU tests (hand-computed convolutions, the
adjoint identity, a band-limited derivative, and the phase of a focused
point diffractor with and without the half-derivative filter).
"""
from __future__ import annotations

import numpy as np


def forward(traces: np.ndarray, taps: np.ndarray, center: int) -> np.ndarray:
    """y[j, n] = sum_k taps[k] x[j, n + center - k] for every trace j (float64)."""
    x = np.asarray(traces, dtype=np.float64)
    h = np.asarray(taps, dtype=np.float64)
    n = x.shape[-1]
    K = h.size
    out = np.empty(x.shape)
    for j in range(x.shape[0]):
        full = np.convolve(x[j], h)  # full[m] = sum_k h[k] x[m - k], m = 0 .. n + K - 2
        out[j] = full[center:center + n] if center + n <= full.size else np.concatenate(
            [full[center:], np.zeros(center + n - full.size)])
    return out


def adjoint(traces: np.ndarray, taps: np.ndarray, center: int) -> np.ndarray:
    """x[j, m] = sum_k taps[k] y[j, m - center + k] for every trace j (float64)."""
    y = np.asarray(traces, dtype=np.float64)
    h = np.asarray(taps, dtype=np.float64)
    n = y.shape[-1]
    K = h.size
    out = np.zeros(y.shape)
    for k in range(K):
        s = k - center  # x[m] += h[k] y[m + s]
        lo, hi = max(0, -s), min(n, n - s)
        if lo < hi:
            out[:, lo:hi] += h[k] * y[:, lo + s:hi + s]
    return out
