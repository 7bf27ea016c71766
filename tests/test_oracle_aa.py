"""Pins of the oracle's anti-alias triangle filter (an operator filter the
paper does not discuss; the production Kirchhoff form is taken: the trace is
smoothed by a unit-area triangle whose half-width p is the time the operator
moves between neighbouring image points, blended linearly between integer
half-widths so that the result is continuous in p).

What pins it without re-typing the oracle: the half-width against the dip of
a hand-computed geometry (a coincident source and receiver at 300 m from a
point 400 m deep: T = 2 * 500 m / v); the impulse response at that geometry
against hand-computed triangle weights; preservation of linear traces (a
symmetric unit-area filter cannot change them); exact equality with the
plain operator when the dip spacing is zero; continuity in p across an
integer half-width; and the FP64 adjoint identity.
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_1204_1225_amd import survey
from tests.test_oracle_pins import hand_problem


def impulse(n_t, m):
    d = np.zeros(n_t, np.float32)
    d[m] = 1.0
    return d


# v = 2000 m/s, dt = 4 ms, s = r at x = 0, point at x = 300 m, z = 400 m:
# T = 2 * 500 / 2000 = 0.5 s -> u = 125 exactly; du/dx = 2 * (300 / 500) / v / dt
# = 0.15 samples per metre.
def aa_point(data, aa, weight=survey.WEIGHT_UNIT):
    p = hand_problem([0.0, 0.0], [0.0, 0.0], [0], data, [300.0], [0.0], [400.0], aperture=60.0, weight=weight)
    return dataclasses.replace(p, aa=aa)


@pytest.mark.parametrize("dx, weights", [
    # p = 0.15 * 20 = 3 (integer): (3 - |k|) / 9
    (20.0, {0: 3 / 9, 1: 2 / 9, 2: 1 / 9, 3: 0.0}),
    # p = 0.15 * 16 = 2.4: 0.6 (2 - |k|)+ / 4 + 0.4 (3 - |k|)+ / 9
    (16.0, {0: 0.6 * 2 / 4 + 0.4 * 3 / 9, 1: 0.6 / 4 + 0.4 * 2 / 9, 2: 0.4 / 9, 3: 0.0}),
    # p = 0.15 * 100 = 15, capped at the largest half-width 3
    (100.0, {0: 3 / 9, 1: 2 / 9, 2: 1 / 9, 3: 0.0}),
    # p = 0.15 * 4 = 0.6 < 1: no smoothing
    (4.0, {0: 1.0, 1: 0.0, 2: 0.0}),
])
def test_impulse_response_closed_form(oracle_lib, dx, weights):
    for k, wk in weights.items():
        for sgn in (1, -1):
            img = oracle_lib.migrate(aa_point(impulse(300, 125 + sgn * k), (dx, 0.0, 3)))
            assert img[0, 0, 0, 0] == pytest.approx(wk, abs=1e-13), (dx, k, sgn)


def test_dip_sums_both_directions(oracle_lib):
    # the point at (300, 0) has no y-dip: any dy leaves p unchanged; a point at
    # (0, 300) has the same dip along y instead.
    d = impulse(300, 126)
    a = oracle_lib.migrate(aa_point(d, (16.0, 0.0, 8)))[0, 0, 0, 0]
    b = oracle_lib.migrate(aa_point(d, (16.0, 50.0, 8)))[0, 0, 0, 0]
    assert a == b and a == pytest.approx(0.6 / 4 + 0.4 * 2 / 9, abs=1e-13)
    q = hand_problem([0.0, 0.0], [0.0, 0.0], [0], d, [0.0], [300.0], [400.0], aperture=60.0,
                     weight=survey.WEIGHT_UNIT)
    c = oracle_lib.migrate(dataclasses.replace(q, aa=(50.0, 16.0, 8)))[0, 0, 0, 0]
    assert c == pytest.approx(a, abs=1e-13)


def test_linear_trace_unchanged(oracle_lib):
    # A linear trace away from the record ends is unchanged by any symmetric
    # unit-area filter, so the anti-aliased image equals the plain one.
    p = survey.make_random(91, n_traces=60, n_t=3000, nx=6, ny=2, nz=30, n_bins=2, dz=10.0, spread=200.0,
                           dt=0.002, data=None)
    k = np.arange(p.n_t, dtype=np.float64)
    p.data = np.tile((0.25 * k - 40.0).astype(np.float32), (p.n_traces, 1))
    plain = oracle_lib.migrate(p)
    aa = oracle_lib.migrate(dataclasses.replace(p, aa=(12.5, 12.5, 6)))
    assert np.abs(aa - plain).max() <= 1e-10 * np.abs(plain).max()


def test_zero_spacing_is_plain_operator(oracle_lib):
    p = survey.make_random(92, n_traces=80, n_t=200, nx=7, ny=3, nz=25, n_bins=2, dz=10.0)
    q = dataclasses.replace(p, aa=(0.0, 0.0, 8))
    assert np.array_equal(oracle_lib.migrate(q), oracle_lib.migrate(p))
    m = np.random.default_rng(3).standard_normal(oracle_lib.migrate(p).shape)
    assert np.array_equal(oracle_lib.demigrate(q, m), oracle_lib.demigrate(p, m))


def test_continuous_in_half_width(oracle_lib):
    # p = 0.15 dx crosses the integer 2 at dx = 13.333..: the value moves by
    # O(step), not by a jump.
    d = np.random.default_rng(5).standard_normal(300).astype(np.float32)
    vals = [oracle_lib.migrate(aa_point(d, (20.0 / 1.5 + e, 0.0, 8)))[0, 0, 0, 0] for e in (-1e-7, 0.0, 1e-7)]
    assert abs(vals[0] - vals[1]) < 1e-5 and abs(vals[2] - vals[1]) < 1e-5


@pytest.mark.parametrize("tf", [0.0, 0.05])
def test_adjoint_identity(oracle_lib, tf):
    p = survey.make_random(93, n_traces=70, n_t=150, nx=8, ny=2, nz=30, n_bins=3, dz=10.0, t_first=tf,
                           data="normal")
    p = dataclasses.replace(p, aa=(12.5, 12.5, 5))
    rng = np.random.default_rng(4)
    d = p.data.astype(np.float64)
    img = oracle_lib.migrate(p)
    m = rng.standard_normal(img.shape)
    lhs = float(np.vdot(img, m))
    rhs = float(np.vdot(d, oracle_lib.demigrate(p, m)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
    smp = np.stack([rng.integers(0, p.n_traces, 40), rng.integers(0, p.n_t, 40)], 1).astype(np.int64)
    full = oracle_lib.demigrate(p, m)
    assert np.allclose(oracle_lib.demigrate_samples(p, m, smp), full[smp[:, 0], smp[:, 1]], rtol=1e-12, atol=1e-12)


def test_smoothing_reaches_past_record_end(oracle_lib):
    # A time just past the last sample still picks up the last samples
    # through the triangle (the plain operator gives 0 there).
    n_t = 120  # u = 125 lies past the record; p = 0.15 * 60 = 9 -> capped at 8
    d = np.ones(n_t, np.float32)
    aa = oracle_lib.migrate(aa_point(d, (60.0, 0.0, 8)))[0, 0, 0, 0]
    plain = oracle_lib.migrate(aa_point(d, None))[0, 0, 0, 0]
    assert plain == 0.0
    # T_8(125) = sum over k with 125 + k <= 119, |k| < 8 of (8 - |k|) / 64 = (1 + 2) / 64
    assert aa == pytest.approx(3 / 64, abs=1e-13)
