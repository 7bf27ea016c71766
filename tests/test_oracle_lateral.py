"""Pins of the oracle's laterally varying table traveltimes: one table
T_n(h, z) per node of a coarse lateral grid, the one-way time interpolated
trilinearly over (image x, image y, h) and taken exactly at the image depths.

Pinned against:
- closed forms: trilinear interpolation reproduces every function in
  span{1, X, Y, h, XY, Xh, Yh, XYh} exactly, so node tables holding such a
  function (dyadic coefficients, exact in float32) give times known in closed
  form at every image point, inside the grid and clamped outside it, for both
  legs of a trace (a swapped axis, a wrong node stride or fraction fails);
- the laterally invariant table path (already pinned against ray tracing,
  hand tables and the double square root): every node holding the same
  table gives that path's image bit for bit;
- the double square root, for constant-velocity tables;
- a diffractor in a laterally varying medium, modelled with curved rays in
  the medium under it and placed on a node whose neighbours hold other media:
  its image there is the closed-form sum of its own modelled samples;
- the adjoint identity."""
import dataclasses

import numpy as np
import pytest

from paper_1204_1225_amd import survey
from tests.test_oracle_pins import hand_problem

# node grid of the hand tables: X = 900, 1000, 1100, 1200; Y = -100, 0, 100 (4 x 3,
# so that a node stride taken along the wrong axis reads other nodes)
GX0, GY0, GD = 900.0, -100.0, 100.0
DH, NH = 50.0, 9  # rows at h = 0, 50, ..., 400 m


def hand_time(X, Y, h, iz):
    """A function in span{1, X, Y, h, XY, Xh, Yh, XYh} (X, Y taken about the
    grid's centre) with dyadic coefficients: exact in float32 on the nodes."""
    a, b = X - 1000.0, Y
    return (0.25 + iz * 2.0 ** -6 + a * 2.0 ** -12 + b * 2.0 ** -13 + h * 2.0 ** -11 + a * b * 2.0 ** -20
            + a * h * 2.0 ** -19 - b * h * 2.0 ** -20 + a * b * h * 2.0 ** -27)


def hand_tables(nz):
    t = np.empty((3, 4, NH, nz), np.float64)
    for j in range(3):
        for i in range(4):
            for ih in range(NH):
                for iz in range(nz):
                    t[j, i, ih, iz] = hand_time(GX0 + i * GD, GY0 + j * GD, ih * DH, iz)
    t32 = t.astype(np.float32)
    assert np.array_equal(t32.astype(np.float64), t)  # exact in float32
    return t32


def clamp(v, lo, hi):
    return min(max(v, lo), hi)


@pytest.mark.parametrize("src,rec", [((1000.0, 0.0), (1000.0, 0.0)), ((1030.0, 20.0), (880.0, -75.0)),
                                     ((700.0, 300.0), (1400.0, 0.0))])
def test_hand_tables_trilinear_closed_form(oracle_lib, src, rec):
    # x and y cross the grid's edges (clamped there), pass through nodes and
    # cell interiors; D[k] = k makes each image value u = (T_s + T_r) / dt.
    x = [850.0, 900.0, 937.5, 1000.0, 1062.5, 1100.0, 1180.0, 1200.0, 1260.0]
    y = [-160.0, -100.0, -37.5, 25.0, 100.0, 140.0]
    z = [100.0, 200.0]
    data = np.arange(800, dtype=np.float32)
    p = hand_problem([src], [rec], [0], data, x, y, z, aperture=89.9, weight=survey.WEIGHT_UNIT)
    p = dataclasses.replace(p, ttab=hand_tables(2), tdh=DH, tgrid=(GX0, GY0, GD, GD))
    img = oracle_lib.migrate(p)
    for iy, py in enumerate(y):
        for ix, px in enumerate(x):
            X, Y = clamp(px, 900.0, 1200.0), clamp(py, -100.0, 100.0)
            for iz in range(2):
                T = 0.0
                for sx, sy in (src, rec):
                    h = float(np.hypot(np.float64(np.float32(px)) - sx, np.float64(np.float32(py)) - sy))
                    T += hand_time(X, Y, min(h, (NH - 1) * DH), iz)
                assert img[0, iy, ix, iz] == pytest.approx(T / 0.004, rel=1e-12, abs=1e-9), (px, py, iz)


def test_single_node_axis(oracle_lib):
    # one node along y (a 2D line): no interpolation in y, x interpolated
    data = np.arange(800, dtype=np.float32)
    tab = hand_tables(1)[1:2]  # the Y = 0 row of nodes, [1][4][n_h][1]
    p = hand_problem([(1010.0, 0.0)], [(960.0, 0.0)], [0], data, [920.0, 1050.0], [0.0], [100.0], aperture=89.9,
                     weight=survey.WEIGHT_UNIT)
    p = dataclasses.replace(p, ttab=tab, tdh=DH, tgrid=(GX0, 1e9, GD, 0.0))
    img = oracle_lib.migrate(p)
    for ix, px in enumerate([920.0, 1050.0]):
        T = hand_time(px, 0.0, abs(px - 1010.0), 0) + hand_time(px, 0.0, abs(px - 960.0), 0)
        assert img[0, 0, ix, 0] == pytest.approx(T / 0.004, rel=1e-12)


def random_table_problem(seed, ny=4):
    p = survey.make_random(seed, n_traces=90, n_t=400, nx=9, ny=ny, nz=40, n_bins=3, dz=10.0, spread=300,
                           weight=survey.WEIGHT_UNIT)
    return survey.with_curved_ray_table(p, dh=5.0)


def test_equal_nodes_give_the_invariant_table_bitwise(oracle_lib):
    pt = random_table_problem(71)
    ref = oracle_lib.migrate(pt)
    tab = np.broadcast_to(pt.ttab, (3, 4) + pt.ttab.shape).copy()
    pl = dataclasses.replace(pt, ttab=tab, tgrid=(950.0, 1950.0, 40.0, 30.0))
    assert np.array_equal(oracle_lib.migrate(pl), ref)
    rng = np.random.default_rng(71)
    m = rng.standard_normal(pt.image_shape)
    assert np.array_equal(oracle_lib.demigrate(pl, m), oracle_lib.demigrate(pt, m))


def test_constant_velocity_lateral_tables_equal_dsr(oracle_lib):
    p = survey.make_random(72, n_traces=100, n_t=400, nx=9, ny=3, nz=50, n_bins=3, dz=10.0,
                           velocity=("const", 2000.0), weight=survey.WEIGHT_UNIT, spread=300)
    ref = oracle_lib.migrate(p)
    pl = survey.with_lateral_tables(p, lambda x, y: 2000.0, 0.0, 900.0, 1900.0, 100.0, 100.0, 4, 5, dh=0.5)
    got = oracle_lib.migrate(pl)
    assert np.linalg.norm(got - ref) <= 2e-4 * np.linalg.norm(ref)


def lateral_diffractor_line():
    # v0(x) = 1500 + 0.25 (x - 1500): the medium under the diffractor is
    # 1500 + 0.5 z; the nodes beside it hold 1437.5 + 0.5 z and 1562.5 + 0.5 z.
    v0_at = survey.lateral_v0(1500.0, 0.25, 0.0, 1500.0, 0.0)
    sx = 50.0 * np.arange(60)
    h = (np.arange(80) - 39.5) * 50.0
    S, H = np.meshgrid(sx, h, indexing="ij")
    src = np.stack([S.ravel(), np.zeros(S.size)], 1)
    rec = np.stack([(S + H).ravel(), np.zeros(S.size)], 1)
    x = 1500.0 + 10.0 * (np.arange(11) - 5)
    z = 10.0 * (np.arange(200) + 1)
    p = survey._finish("lateral_line", src, rec, 1000, 0.004, 0.0, x, [0.0], z, 4, 500.0, ("linear", 1500.0, 0.5),
                       60.0, weight=survey.WEIGHT_UNIT)
    p.scatterers = np.array([[1500.0, 0.0, 1500.0]])
    p.data = survey.model_scatterers(p, p.scatterers, rays="curved", v0_at=v0_at).numpy()
    return p, v0_at


def test_lateral_diffractor_image_at_its_node(oracle_lib):
    p, v0_at = lateral_diffractor_line()
    pl = survey.with_lateral_tables(p, v0_at, 0.5, 1250.0, 0.0, 250.0, 1.0, 3, 1, dh=2.0)
    img = oracle_lib.migrate(pl)
    ix, iz = 5, 149  # x = 1500 (node 1), z = 1500
    hs = np.abs(p.src[:, 0].astype(np.float64) - 1500.0)
    hr = np.abs(p.rec[:, 0].astype(np.float64) - 1500.0)
    tau = survey.curved_ray_time(hs, 1500.0, 1500.0, 0.5) + survey.curved_ray_time(hr, 1500.0, 1500.0, 0.5)
    r2 = float(p.r2[iz])
    inside = (hs * hs <= r2) & (hr * hr <= r2)
    for b in range(p.n_bins):
        sel = inside & (p.bin == b)
        u = tau[sel] / p.dt
        i = np.floor(u).astype(np.int64)
        f = u - i
        d = p.data[sel].astype(np.float64)
        rows = np.arange(d.shape[0])
        expect = float(np.sum((1 - f) * d[rows, i] + f * d[rows, i + 1]))
        assert img[b, 0, ix, iz] == pytest.approx(expect, rel=2e-5)
    # the neighbouring nodes' media do not focus it: a table built on either
    # one alone puts much less energy there
    for v0 in (1437.5, 1562.5):
        pw = survey.with_lateral_tables(p, lambda x, y, v=v0: v, 0.5, 1250.0, 0.0, 250.0, 1.0, 3, 1, dh=2.0)
        assert img[3, 0, ix, iz] > 1.5 * abs(oracle_lib.migrate(pw)[3, 0, ix, iz])


def test_lateral_table_adjoint_identity(oracle_lib):
    p = survey.make_random(73, n_traces=80, n_t=300, nx=7, ny=4, nz=40, n_bins=2, dz=10.0, spread=300)
    pl = survey.with_lateral_tables(p, survey.lateral_v0(1500.0, 0.2, -0.1, 1000.0, 2000.0), 0.5, 960.0, 1970.0,
                                    40.0, 30.0, 3, 3, dh=5.0)
    rng = np.random.default_rng(73)
    d = rng.standard_normal((pl.n_traces, pl.n_t))
    m = rng.standard_normal(pl.image_shape)
    lhs = float(np.sum(oracle_lib.migrate(pl, data=d) * m))
    rhs = float(np.sum(d * oracle_lib.demigrate(pl, m)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))


def test_lateral_grid_validation(oracle_lib):
    pt = random_table_problem(74)
    tab = np.broadcast_to(pt.ttab, (2, 2) + pt.ttab.shape).copy()
    for grid in [(0.0, 0.0, 0.0, 10.0), (0.0, 0.0, 10.0, -1.0)]:
        with pytest.raises(ValueError):
            oracle_lib.migrate(dataclasses.replace(pt, ttab=tab, tgrid=grid))
