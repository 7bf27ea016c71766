"""Pins of the trace pre-filter oracle (oracle/trace_filter.py) and of the
rho-filter taps of the input generator.

Hand-computed convolutions, the adjoint identity, shifts, the band-limited
derivative the alpha = 1 taps must reproduce, and the physics the filter is
for: the constant-velocity migration of a flat reflector is a summation over
a traveltime surface that lies later than its apex, which rotates the wavelet
by about +45 degrees on a line; the alpha = 1/2 pre-filter returns it to zero
phase at every offset (measured on the analytic signal at the envelope peak).
"""
import numpy as np
import pytest
from scipy.signal import hilbert

from oracle import trace_filter as tf
from paper_1204_1225_amd import survey


def test_hand_convolution_and_transpose():
    taps = np.array([1.0, 2.0, 3.0])
    x = np.array([[1.0, 0.0, 0.0, 1.0, 0.0]])
    assert tf.forward(x, taps, 1)[0].tolist() == [2.0, 3.0, 1.0, 2.0, 3.0]
    e2 = np.array([[0.0, 0.0, 1.0, 0.0, 0.0]])
    assert tf.adjoint(e2, taps, 1)[0].tolist() == [0.0, 3.0, 2.0, 1.0, 0.0]


@pytest.mark.parametrize("K,c", [(1, 0), (5, 0), (5, 4), (7, 3), (40, 17)])
def test_delta_taps_shift(K, c):
    rng = np.random.default_rng(K + c)
    x = rng.standard_normal((3, 30))
    for j in range(K):
        taps = np.zeros(K)
        taps[j] = 1.0
        y = tf.forward(x, taps, c)
        s = c - j  # y[n] = x[n + s]
        ref = np.zeros_like(x)
        lo, hi = max(0, -s), min(30, 30 - s)
        if lo < hi:
            ref[:, lo:hi] = x[:, lo + s:hi + s]
        assert np.array_equal(y, ref)


@pytest.mark.parametrize("K,c,n", [(9, 4, 50), (3, 0, 7), (64, 63, 20), (65, 32, 200)])
def test_adjoint_identity(K, c, n):
    rng = np.random.default_rng(n)
    taps = rng.standard_normal(K)
    x = rng.standard_normal((4, n))
    y = rng.standard_normal((4, n))
    lhs = float(np.sum(tf.forward(x, taps, c) * y))
    rhs = float(np.sum(x * tf.adjoint(y, taps, c)))
    assert abs(lhs - rhs) <= 1e-12 * np.sqrt(np.sum(x * x) * np.sum(y * y)) * np.abs(taps).sum()


def test_alpha_one_taps_are_minus_derivative():
    t = np.arange(2000) * 0.004
    taps, c = survey.rho_filter_taps(0.004, 1.0, half_len=48)
    for f in (10.0, 20.0, 40.0):
        y = tf.forward(np.cos(2 * np.pi * f * t)[None, :], taps, c)[0, 200:-200]
        ref = (2 * np.pi * f * np.sin(2 * np.pi * f * t))[200:-200]
        assert np.abs(y - ref).max() <= 1e-4 * np.abs(ref).max()


def test_half_derivative_zero_phases_flat_reflector(oracle_lib):
    p = survey.make_flat_line()
    taps, c = survey.rho_filter_taps(p.dt, 0.5)
    for data, want, tol in [(p.data, 45.0, 5.0), (tf.forward(p.data, taps, c), 0.0, 3.0)]:
        img = oracle_lib.migrate(p, data=np.asarray(data, np.float64))
        for b in range(p.n_bins):
            a = hilbert(img[b, 0, 2])
            k = int(np.argmax(np.abs(a)))
            assert p.z[k] == pytest.approx(800.0, abs=5.0)
            assert abs(np.degrees(np.angle(a[k])) - want) < tol
