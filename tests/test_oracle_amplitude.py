"""Pins of the oracle's amplitude tables for table traveltimes: a one-way
amplitude A per leg, interpolated exactly as the time is (linear in h; for
laterally varying tables also in x and y), and W = A_s A_r in place of W = 1.

Pinned against:
- the square-root form's cos cos / (T_s T_r) weight, which for constant
  velocity is the product of the legs' t0 / T^2 (to the tables' interpolation
  error);
- closed forms: hand amplitude tables linear in h (one trace, D[k] = k, so the
  image value is u A_s A_r), and on a lateral node grid a function in
  span{1, X, Y, h, XY, Xh, Yh, XYh}, reproduced exactly by the interpolation;
- amplitudes of 1: the unit weight bit for bit;
- the adjoint identity."""
import dataclasses

import numpy as np
import pytest

from paper_1204_1225_amd import survey
from tests.test_oracle_lateral import DH, GD, GX0, GY0, NH, clamp, hand_tables, hand_time
from tests.test_oracle_pins import hand_problem


def test_constant_velocity_amplitudes_give_the_coscos_weight(oracle_lib):
    p = survey.make_random(91, n_traces=100, n_t=400, nx=9, ny=3, nz=50, n_bins=3, dz=10.0,
                           velocity=("const", 2000.0), weight=survey.WEIGHT_COSCOS, spread=300)
    ref = oracle_lib.migrate(p)
    pt = survey.with_curved_ray_table(p, dh=0.5, amplitude=True)
    got = oracle_lib.migrate(pt)
    assert np.linalg.norm(got - ref) <= 2e-4 * np.linalg.norm(ref)
    # without the amplitudes the images differ by the weight itself
    plain = oracle_lib.migrate(survey.with_curved_ray_table(p, dh=0.5))
    assert np.linalg.norm(plain - ref) > 0.5 * np.linalg.norm(ref)
    pl = survey.with_lateral_tables(p, lambda x, y: 2000.0, 0.0, 900.0, 1900.0, 100.0, 100.0, 3, 4, dh=0.5,
                                    amplitude=True)
    assert np.linalg.norm(oracle_lib.migrate(pl) - ref) <= 2e-4 * np.linalg.norm(ref)


def test_unit_amplitudes_are_the_unit_weight(oracle_lib):
    p = survey.make_random(92, n_traces=80, n_t=300, nx=7, ny=4, nz=40, n_bins=2, dz=10.0, spread=300)
    pt = survey.with_curved_ray_table(p, dh=5.0)
    ones = dataclasses.replace(pt, tamp=np.ones_like(pt.ttab))
    assert np.array_equal(oracle_lib.migrate(ones), oracle_lib.migrate(pt))
    m = np.random.default_rng(92).standard_normal(pt.image_shape)
    assert np.array_equal(oracle_lib.demigrate(ones, m), oracle_lib.demigrate(pt, m))


def test_hand_amplitude_rows(oracle_lib):
    # time rows 0.125 s and 0.25 s at h = 0 and 100 m; amplitude rows 2 and 3
    # (exact in float32): at leg length h, A = 2 + h / 100 up to the last row.
    data = np.arange(400, dtype=np.float32)
    for hs, hr in [(0.0, 0.0), (50.0, 25.0), (100.0, 75.0), (30.0, 250.0)]:
        p = hand_problem([1000.0 - hs, 0.0], [1000.0 + hr, 0.0], [0], data, [1000.0], [0.0], [300.0],
                         aperture=89.0, weight=survey.WEIGHT_UNIT)
        p = dataclasses.replace(p, ttab=np.array([[0.125], [0.25]], np.float32), tdh=100.0,
                                tamp=np.array([[2.0], [3.0]], np.float32))

        def lerp(h, a, b):
            f = min(h / 100.0, 1.0)
            return a + f * (b - a)

        u = (lerp(hs, 0.125, 0.25) + lerp(hr, 0.125, 0.25)) / 0.004
        w = lerp(hs, 2.0, 3.0) * lerp(hr, 2.0, 3.0)
        assert oracle_lib.migrate(p)[0, 0, 0, 0] == pytest.approx(u * w, rel=1e-12)


def hand_amp(X, Y, h, iz):
    """Another function in span{1, X, Y, h, XY, Xh, Yh, XYh}, positive on the
    grid, dyadic coefficients."""
    a, b = X - 1000.0, Y
    return (1.5 + iz * 2.0 ** -4 - a * 2.0 ** -9 + b * 2.0 ** -10 + h * 2.0 ** -10 + a * b * 2.0 ** -17
            - a * h * 2.0 ** -16 + b * h * 2.0 ** -18 + a * b * h * 2.0 ** -25)


def hand_amp_tables(nz):
    t = np.empty((3, 4, NH, nz), np.float64)
    for j in range(3):
        for i in range(4):
            for ih in range(NH):
                for iz in range(nz):
                    t[j, i, ih, iz] = hand_amp(GX0 + i * GD, GY0 + j * GD, ih * DH, iz)
    t32 = t.astype(np.float32)
    assert np.array_equal(t32.astype(np.float64), t)
    return t32


@pytest.mark.parametrize("src,rec", [((1030.0, 20.0), (880.0, -75.0)), ((700.0, 300.0), (1400.0, 0.0))])
def test_lateral_amplitudes_closed_form(oracle_lib, src, rec):
    x = [850.0, 937.5, 1000.0, 1062.5, 1180.0, 1260.0]
    y = [-160.0, -37.5, 25.0, 100.0, 140.0]
    z = [100.0, 200.0]
    data = np.arange(800, dtype=np.float32)
    p = hand_problem([src], [rec], [0], data, x, y, z, aperture=89.9, weight=survey.WEIGHT_UNIT)
    p = dataclasses.replace(p, ttab=hand_tables(2), tamp=hand_amp_tables(2), tdh=DH, tgrid=(GX0, GY0, GD, GD))
    img = oracle_lib.migrate(p)
    for iy, py in enumerate(y):
        for ix, px in enumerate(x):
            X, Y = clamp(px, 900.0, 1200.0), clamp(py, -100.0, 100.0)
            for iz in range(2):
                T, W = 0.0, 1.0
                for sx, sy in (src, rec):
                    h = float(np.hypot(np.float64(np.float32(px)) - sx, np.float64(np.float32(py)) - sy))
                    hc = min(h, (NH - 1) * DH)
                    T += hand_time(X, Y, hc, iz)
                    W *= hand_amp(X, Y, hc, iz)
                assert img[0, iy, ix, iz] == pytest.approx(T / 0.004 * W, rel=1e-12), (px, py, iz)


@pytest.mark.parametrize("lateral", [False, True])
def test_amplitude_adjoint_identity(oracle_lib, lateral):
    p = survey.make_random(93, n_traces=80, n_t=300, nx=7, ny=4, nz=40, n_bins=2, dz=10.0, spread=300)
    if lateral:
        pa = survey.with_lateral_tables(p, survey.lateral_v0(1500.0, 0.2, -0.1, 1000.0, 2000.0), 0.5, 960.0,
                                        1970.0, 40.0, 30.0, 3, 3, dh=5.0, amplitude=True)
    else:
        pa = survey.with_curved_ray_table(p, dh=5.0, amplitude=True)
    rng = np.random.default_rng(93)
    d = rng.standard_normal((pa.n_traces, pa.n_t))
    m = rng.standard_normal(pa.image_shape)
    lhs = float(np.sum(oracle_lib.migrate(pa, data=d) * m))
    rhs = float(np.sum(d * oracle_lib.demigrate(pa, m)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))
