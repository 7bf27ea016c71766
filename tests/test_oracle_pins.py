"""Pins of the FP64 oracle against what Eq. (1) and Eq. (2) fix.

Nothing here re-types the oracle's formula: the expectations are closed-form
values derived by hand for single traces (exact Pythagorean geometries),
invariants of the integral (linearity, source/receiver reciprocity, the
summation form behind the Map/Reduce decomposition of Section 4, offset-bin
partition, translation), the adjoint identity, the isochron of the textbook
diffraction stack written with Euclidean distances, an integer count of the
45-degree aperture cone, and the focusing of point diffractors by
constructive interference (Section 3).
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_1204_1225_amd import survey


def hand_problem(src, rec, bins, data, x, y, z, v=2000.0, aperture=45.0, t_first=0.0, dt=0.004,
                 weight=survey.WEIGHT_COSCOS, n_bins=None, velocity=None):
    src = np.asarray(src, np.float32).reshape(-1, 2)
    rec = np.asarray(rec, np.float32).reshape(-1, 2)
    z = np.asarray(z, np.float64)
    vel = velocity or ("const", v)
    t0sq, s2 = survey.traveltime_tables(z, vel)
    data = np.asarray(data, np.float32).reshape(src.shape[0], -1)
    return survey.Problem(name="hand", src=src, rec=rec, bin=np.asarray(bins, np.int32), data=data,
                          n_t=data.shape[1], dt=dt, t_first=t_first, x=np.asarray(x, np.float32),
                          y=np.asarray(y, np.float32), z=z, n_bins=n_bins or (int(max(bins)) + 1),
                          t0sq=t0sq, s2=s2, r2=survey.aperture_table(t0sq, s2, aperture), weight=weight,
                          velocity=vel, aperture_deg=aperture)


def quad_trace(n_t=400):
    """D[k] = k^2 + 1: linear interpolation at u = i + f gives i^2 + 1 + f (2 i + 1)."""
    k = np.arange(n_t, dtype=np.float64)
    return (k * k + 1.0).astype(np.float32)


def lerp_quad(u):
    i = math.floor(u)
    f = u - i
    return i * i + 1.0 + f * (2 * i + 1)


REL = 1e-12


# --------------------------------------------------------------------------
# Closed forms: one trace, one image column, constant v = 2000 m/s, dt = 4 ms
# --------------------------------------------------------------------------

def test_zero_offset_on_sample(oracle_lib):
    # s = r directly above the point, z = 400 m: T = 2 * 0.2 s -> u = 100;
    # W = cos*cos/(Ts*Tr) = 1 / 0.2^2 = 25.
    p = hand_problem([1000, 0], [1000, 0], [0], quad_trace(), [1000.0], [0.0], [400.0])
    img = oracle_lib.migrate(p)
    assert img.shape == (1, 1, 1, 1)
    assert img[0, 0, 0, 0] == pytest.approx(25.0 * (100 ** 2 + 1), rel=REL)


def test_zero_offset_half_sample(oracle_lib):
    # z = 402 m: T = 0.402 s -> u = 100.5, W = (v / z)^2.
    p = hand_problem([1000, 0], [1000, 0], [0], quad_trace(), [1000.0], [0.0], [402.0])
    w = (2000.0 / 402.0) ** 2
    assert oracle_lib.migrate(p)[0, 0, 0, 0] == pytest.approx(w * lerp_quad(100.5), rel=REL)


def test_split_spread_345(oracle_lib):
    # Source and receiver 300 m either side, z = 400 m: each leg 500 m (3-4-5),
    # Ts = Tr = 0.25 s -> u = 125; cos = 0.8 -> W = 0.64 / 0.0625 = 10.24.
    p = hand_problem([700, 0], [1300, 0], [0], quad_trace(), [1000.0], [0.0], [400.0])
    assert oracle_lib.migrate(p)[0, 0, 0, 0] == pytest.approx(10.24 * (125 ** 2 + 1), rel=REL)


def test_asymmetric_legs(oracle_lib):
    # Source leg 500 m (0.25 s), receiver leg vertical 400 m (0.2 s): u = 112.5,
    # W = (0.8 / 0.25) * (1 / 0.2) = 16.
    p = hand_problem([700, 0], [1000, 0], [0], quad_trace(), [1000.0], [0.0], [400.0])
    assert oracle_lib.migrate(p)[0, 0, 0, 0] == pytest.approx(16.0 * lerp_quad(112.5), rel=REL)


def test_unit_weight(oracle_lib):
    p = hand_problem([700, 0], [1300, 0], [0], quad_trace(), [1000.0], [0.0], [400.0],
                     weight=survey.WEIGHT_UNIT)
    assert oracle_lib.migrate(p)[0, 0, 0, 0] == pytest.approx(125 ** 2 + 1, rel=REL)


def test_t_first_shift(oracle_lib):
    # Record starts at 0.1 s: u = (0.4 - 0.1) / 0.004 = 75.
    p = hand_problem([1000, 0], [1000, 0], [0], quad_trace(), [1000.0], [0.0], [400.0], t_first=0.1)
    assert oracle_lib.migrate(p)[0, 0, 0, 0] == pytest.approx(25.0 * (75 ** 2 + 1), rel=REL)


def test_record_ends(oracle_lib):
    w = (2000.0 / 402.0) ** 2
    # u = 100.5 with 101 samples: only (1 - f) D[100] survives.
    p = hand_problem([1000, 0], [1000, 0], [0], quad_trace(101), [1000.0], [0.0], [402.0])
    assert oracle_lib.migrate(p)[0, 0, 0, 0] == pytest.approx(w * 0.5 * (100 ** 2 + 1), rel=REL)
    # u = 100 with 100 samples: outside the record.
    p = hand_problem([1000, 0], [1000, 0], [0], quad_trace(100), [1000.0], [0.0], [400.0])
    assert oracle_lib.migrate(p)[0, 0, 0, 0] == 0.0
    # u = -0.25 (record starts at 0.401 s): f = 0.75 of D[0] = 1.
    p = hand_problem([1000, 0], [1000, 0], [0], quad_trace(), [1000.0], [0.0], [400.0], t_first=0.401)
    assert oracle_lib.migrate(p)[0, 0, 0, 0] == pytest.approx(25.0 * 0.75, rel=1e-9)
    # u = -1.25: nothing.
    p = hand_problem([1000, 0], [1000, 0], [0], quad_trace(), [1000.0], [0.0], [400.0], t_first=0.405)
    assert oracle_lib.migrate(p)[0, 0, 0, 0] == 0.0


def test_aperture_edge_inclusive(oracle_lib):
    # 45 degrees: both legs at h = z = 400 m are inside (h^2 <= r2 = z^2).
    p = hand_problem([600, 0], [600, 0], [0], quad_trace(), [1000.0], [0.0], [400.0])
    T = 2 * math.hypot(400.0, 400.0) / 2000.0
    w = 0.04 / (T / 2) ** 4
    assert oracle_lib.migrate(p)[0, 0, 0, 0] == pytest.approx(w * lerp_quad(T / 0.004), rel=1e-11)
    # 1 cm further out on one leg only: outside.
    p = hand_problem([599.99, 0], [600, 0], [0], quad_trace(), [1000.0], [0.0], [400.0])
    assert oracle_lib.migrate(p)[0, 0, 0, 0] == 0.0
    p = hand_problem([600, 0], [1400.01, 0], [0], quad_trace(), [1000.0], [0.0], [400.0])
    assert oracle_lib.migrate(p)[0, 0, 0, 0] == 0.0


def test_3d_layout_and_crossline_leg(oracle_lib):
    # 3 x 2 columns, two depths, two bins.  Trace 0 (bin 1) is a crossline
    # split spread of 300 m around column (x=1010, y=2000): only image
    # I[1, iy=1, ix=1, iz=1] (z = 400) sees the 3-4-5 geometry at u = 125.
    x = [1000.0, 1010.0, 1020.0]
    y = [1990.0, 2000.0]
    z = [390.0, 400.0]
    d = np.stack([np.zeros(400, np.float32), quad_trace()])
    p = hand_problem([[0, -1e6], [1010, 1700]], [[0, -1e6], [1010, 2300]], [0, 1], d, x, y, z, n_bins=2)
    img = oracle_lib.migrate(p)
    assert img.shape == (2, 2, 3, 2)
    assert img[1, 1, 1, 1] == pytest.approx(10.24 * (125 ** 2 + 1), rel=REL)
    assert np.all(img[0] == 0.0)
    # the neighbouring columns see a longer path: strictly later samples
    assert img[1, 1, 0, 1] != img[1, 1, 1, 1]


def test_bin_selects_traces(oracle_lib):
    # A trace only images into its own offset bin; an out-of-range bin is unused.
    d = np.stack([quad_trace(), quad_trace()])
    p = hand_problem([[1000, 0], [1000, 0]], [[1000, 0], [1000, 0]], [0, 2], d, [1000.0], [0.0], [400.0],
                     n_bins=2)
    img = oracle_lib.migrate(p)
    assert img[0, 0, 0, 0] == pytest.approx(25.0 * (100 ** 2 + 1), rel=REL)
    assert img[1, 0, 0, 0] == 0.0


def test_diffraction_stack_isochron(oracle_lib):
    # Textbook special case: W = 1, constant v, no aperture limit, one spike
    # at sample n0.  Each image point sees the spike through the hat function
    # of (u - n0), with u from the Euclidean source and receiver path lengths.
    nt, n0 = 600, 150
    d = np.zeros(nt, np.float32)
    d[n0] = 1.0
    x = 1000.0 + 10.0 * np.arange(-30, 31)
    z = 10.0 * (np.arange(80) + 1)
    p = hand_problem([850, 0], [1120, 0], [0], d, x, [0.0], z, aperture=90.0, weight=survey.WEIGHT_UNIT)
    img = oracle_lib.migrate(p)[0, 0]
    X, Z = np.meshgrid(x.astype(np.float64), z, indexing="ij")
    u = (np.hypot(X - 850.0, Z) + np.hypot(X - 1120.0, Z)) / 2000.0 / 0.004
    expect = np.maximum(0.0, 1.0 - np.abs(u - n0))
    assert np.max(np.abs(img - expect)) < 1e-9
    assert np.count_nonzero(expect) > 50


# --------------------------------------------------------------------------
# Invariants of Eq. (1)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small():
    return survey.make_random(11, n_traces=150, n_t=300, nx=9, ny=7, nz=40, n_bins=3, dz=20.0)


def test_linearity(oracle_lib, small):
    d1 = small.data.astype(np.float64)
    d2 = survey.random_data(small, 99).astype(np.float64)
    a, b = 0.7, -1.3
    lhs = oracle_lib.migrate(small, a * d1 + b * d2)
    rhs = a * oracle_lib.migrate(small, d1) + b * oracle_lib.migrate(small, d2)
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(rhs)


def test_reciprocity(oracle_lib, small):
    import dataclasses

    sw = dataclasses.replace(small, src=small.rec.copy(), rec=small.src.copy())
    assert np.array_equal(oracle_lib.migrate(small), oracle_lib.migrate(sw))


def test_trace_partition_summation_form(oracle_lib, small):
    # Map per trace, Reduce = sum (Section 4): migrating shards and summing
    # their images equals migrating everything.
    full = oracle_lib.migrate(small)
    rng = np.random.default_rng(5)
    lab = rng.integers(0, 4, small.n_traces)
    acc = np.zeros_like(full)
    for k in range(4):
        acc += oracle_lib.migrate(small.subset(np.nonzero(lab == k)[0]))
    assert np.linalg.norm(acc - full) <= 1e-13 * np.linalg.norm(full)
    # Map at the finest grain: one trace per map task.
    idx = np.arange(12)
    per_trace = sum(oracle_lib.migrate(small.subset([j])) for j in idx)
    ref = oracle_lib.migrate(small.subset(idx))
    assert np.count_nonzero(ref) > 0
    assert np.linalg.norm(per_trace - ref) <= 1e-13 * np.linalg.norm(ref)


def test_bin_partition(oracle_lib, small):
    import dataclasses

    merged = dataclasses.replace(small, bin=np.zeros_like(small.bin), n_bins=1)
    assert np.allclose(oracle_lib.migrate(small).sum(0), oracle_lib.migrate(merged)[0], rtol=0, atol=1e-12 *
                       np.abs(oracle_lib.migrate(merged)).max())


def test_translation(oracle_lib):
    import dataclasses

    p = survey.make_line2d(1)
    p = p.subset(np.arange(0, p.n_traces, 7))
    sh = np.float32(1024.0)
    q = dataclasses.replace(p, src=p.src + np.array([sh, 0], np.float32), rec=p.rec + np.array([sh, 0], np.float32),
                            x=p.x + sh)
    assert np.array_equal(oracle_lib.migrate(p), oracle_lib.migrate(q))


def test_adjoint_dot_product(oracle_lib, small):
    d = survey.random_data(small, 41).astype(np.float64)
    m = survey.random_image(small, 42).astype(np.float64)
    lhs = float(np.vdot(oracle_lib.migrate(small, d), m))
    rhs = float(np.vdot(d, oracle_lib.demigrate(small, m)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))


def test_adjoint_spike_closed_form(oracle_lib):
    # Image spike at (z = 402) under a zero-offset trace: the adjoint splits
    # W * m into samples 100 and 101 with weights 0.5 / 0.5.
    p = hand_problem([1000, 0], [1000, 0], [0], np.zeros(200, np.float32), [1000.0], [0.0], [402.0])
    d = oracle_lib.demigrate(p, np.full((1, 1, 1, 1), 2.0))
    w = (2000.0 / 402.0) ** 2
    assert d[0, 100] == pytest.approx(0.5 * w * 2.0, rel=REL)
    assert d[0, 101] == pytest.approx(0.5 * w * 2.0, rel=REL)
    assert np.count_nonzero(d) == 2


def test_window_is_columns_restricted(oracle_lib, small):
    # a depth window of columns is the same sum, depth by depth (bit for bit:
    # same pair evaluations added in the same trace order)
    cols = np.array([[0, 0, 0], [1, 3, 4], [2, 6, 8], [0, 5, 2]], np.int32)
    full = oracle_lib.migrate_columns(small, cols)
    for z_lo, z_hi in [(0, 40), (7, 23), (39, 40), (12, 12)]:
        assert np.array_equal(oracle_lib.migrate_window(small, cols, z_lo, z_hi), full[:, z_lo:z_hi])
    with pytest.raises(ValueError):
        oracle_lib.migrate_window(small, cols, 30, 41)


def test_pointwise_entry_points_agree(oracle_lib, small):
    full = oracle_lib.migrate(small)
    pts = np.array([[b, iy, ix, iz] for b, iy, ix, iz in [(0, 3, 4, 39), (2, 0, 8, 10), (1, 6, 0, 25)]])
    assert np.allclose(oracle_lib.migrate_points(small, pts), full[tuple(pts.T)], rtol=1e-13, atol=0)
    cols = np.array([[1, 2, 3], [2, 6, 8]])
    assert np.allclose(oracle_lib.migrate_columns(small, cols), full[cols[:, 0], cols[:, 1], cols[:, 2]],
                       rtol=1e-13, atol=0)
    m = survey.random_image(small, 3).astype(np.float64)
    dfull = oracle_lib.demigrate(small, m)
    smp = np.array([[0, 100], [37, 250], [149, 3], [80, 299]])
    assert np.allclose(oracle_lib.demigrate_samples(small, m, smp), dfull[smp[:, 0], smp[:, 1]], rtol=1e-12,
                       atol=1e-12 * np.abs(dfull).max())


def test_count_45_degree_cone(oracle_lib):
    # One zero-offset trace at x = 1000, image x = 1000 + 10 k (k = -50..50),
    # z = 10 (iz + 1): inside iff |x - 1000| <= z, so each depth holds
    # 2 min(iz + 1, 50) + 1 columns.
    x = 1000.0 + 10.0 * np.arange(-50, 51)
    z = 10.0 * (np.arange(200) + 1)
    p = hand_problem([1000, 0], [1000, 0], [0], np.zeros(5000, np.float32), x, [0.0], z)
    na, ne = oracle_lib.count(p)
    expect = sum(2 * min(iz + 1, 50) + 1 for iz in range(200))
    assert na == expect
    assert ne == expect  # 5000 samples reach past every diagonal time
    p.n_t = 10
    p.data = np.zeros((1, 10), np.float32)
    na2, ne2 = oracle_lib.count(p)
    assert na2 == expect and ne2 < na2


def exact_time_problem(n_t, t_first=0.0, n_depths=16):
    # One zero-offset trace straight above one image column.  v = 1024 m/s,
    # dt = 1/256 s and depths z = 512 + k m make every time exact in binary:
    # t0 = z / 1024, T_s + T_r = 2 t0, u = (2 t0 - t_first) / dt = 256 + k/2 -
    # t_first/dt, with no rounding anywhere (squares of dyadic rationals, exact
    # square roots).  h = 0, so every depth is inside the aperture.
    z = 512.0 + np.arange(n_depths)
    return hand_problem([1000, 0], [1000, 0], [0], np.zeros(n_t, np.float32), [1000.0], [0.0], z, v=1024.0,
                        dt=1.0 / 256.0, t_first=t_first)


@pytest.mark.parametrize("n_t,t_first,expect_eff", [
    # u_k = 256 + k/2 (k = 0..15)
    (260, 0.0, 8),             # k = 8 gives u = 260 = N_t exactly: excluded; k = 0..7 inside
    (261, 0.0, 10),            # k = 9 gives u = 260.5 in (N_t - 1, N_t): included
    (257, 0.0, 2),             # u = 256 = N_t - 1 (the last sample, f = 0) and 256.5: included
    (256, 0.0, 0),             # u = 256 = N_t: excluded
    (1000, 258.0 / 256.0, 13),  # u_k = k/2 - 2: k = 2 gives u = -1 exactly (excluded), k = 3 gives -0.5
    (1000, 257.5 / 256.0, 14),  # u_k = k/2 - 1.5: k = 1 gives -1 (excluded), k = 2 gives -0.5 (included)
])
def test_count_effective_at_record_ends(oracle_lib, n_t, t_first, expect_eff):
    # n_effective counts the pairs with -1 < u < N_t (Eq. (2)'s traces whose
    # time falls where the zero-extended record has a sample that can be
    # nonzero); the aperture count does not depend on the record.
    p = exact_time_problem(n_t, t_first)
    na, ne = oracle_lib.count(p)
    assert na == 16
    assert ne == expect_eff
    assert oracle_lib.count_columns(p, [[0, 0, 0]]) == (16, expect_eff)


def test_count_effective_values_are_the_interpolated_ones(oracle_lib):
    # The pairs counted as effective are exactly those whose migrated value can
    # be nonzero: with D = 1 everywhere, the image at depth k is the weight
    # times (1 - f) D[i] + f D[i + 1] on the zero-extended record, which is 0
    # iff u <= -1 or u >= N_t.
    p = exact_time_problem(261, 258.5 / 256.0)  # u_k = k/2 - 2.5: k = 3 gives -1, k = 4 gives -0.5
    p.data = np.ones((1, 261), np.float32)
    p.weight = survey.WEIGHT_UNIT
    img = oracle_lib.migrate(p)[0, 0, 0]
    _, ne = oracle_lib.count(p)
    assert ne == int(np.count_nonzero(img)) == 12
    assert img[3] == 0.0 and img[4] == pytest.approx(0.5, rel=REL)


def test_count_columns_cone_by_hand(oracle_lib):
    # The 45-degree cone of test_count_45_degree_cone split by image column:
    # column x = 1000 + 10 k holds depth iz iff 10 |k| <= 10 (iz + 1), i.e.
    # 200 - max(|k| - 1, 0) of the 200 depths; with N_t = 100 (u = 2.5
    # sqrt((iz + 1)^2 + k^2) samples at v = 2000 m/s, dt = 4 ms) the pairs with
    # (iz + 1)^2 + k^2 < 1600 are effective (integer arithmetic below).
    x = 1000.0 + 10.0 * np.arange(-50, 51)
    z = 10.0 * (np.arange(200) + 1)
    p = hand_problem([1000, 0], [1000, 0], [0], np.zeros(100, np.float32), x, [0.0], z)
    for k in [-50, -37, -3, -1, 0, 1, 2, 29, 50]:
        ix = k + 50
        exp_ap = 200 - max(abs(k) - 1, 0)
        exp_eff = sum(1 for iz in range(200) if iz + 1 >= abs(k) and (iz + 1) ** 2 + k * k < 1600)
        assert oracle_lib.count_columns(p, [[0, 0, ix]]) == (exp_ap, exp_eff), k
    # a column of another bin holds none of this bin-0 trace's pairs
    p.n_bins = 2
    assert oracle_lib.count_columns(p, [[1, 0, 50]]) == (0, 0)


def test_count_columns_sum_to_count(oracle_lib, small):
    # Summed over every image column of every bin, the per-column counts are
    # the total counts (one evaluation path per column against all traces of
    # its bin versus one per trace against all columns of its bin).
    p = dataclasses.replace(small, n_t=120, t_first=0.03)
    cols = np.array([(b, iy, ix) for b in range(p.n_bins) for iy in range(len(p.y)) for ix in range(len(p.x))],
                    dtype=np.int32)
    na, ne = oracle_lib.count(p)
    assert oracle_lib.count_columns(p, cols) == (na, ne)
    assert 0 < ne < na
    half = cols[: len(cols) // 2]
    a = oracle_lib.count_columns(p, half)
    b = oracle_lib.count_columns(p, cols[len(cols) // 2:])
    assert (a[0] + b[0], a[1] + b[1]) == (na, ne)


# --------------------------------------------------------------------------
# Focusing (Section 3: constructive interference builds the reflectors)
# --------------------------------------------------------------------------

def test_focusing_line2d(oracle_lib):
    p = survey.make_line2d(1)
    stack = oracle_lib.migrate(p).sum(0)[0]  # [nx, nz]
    for ix, _, iz in p.diffractor_nodes:
        win = np.abs(stack[ix - 5:ix + 6, iz - 5:iz + 6])
        assert np.unravel_index(np.argmax(win), win.shape) == (5, 5)


# --------------------------------------------------------------------------
# Input-generator pins (traveltime tables, bins, storage conversion)
# --------------------------------------------------------------------------

def test_rms_tables_by_quadrature():
    from scipy.integrate import quad

    v0, k = 1500.0, 0.5
    z = np.array([5.0, 400.0, 1234.0, 2000.0])
    t0sq, s2 = survey.traveltime_tables(z, ("linear", v0, k))
    for i, zz in enumerate(z):
        t0 = quad(lambda s: 1.0 / (v0 + k * s), 0.0, zz, epsabs=0, epsrel=1e-13)[0]
        # v as a function of vertical time: z(t) solves dz/dt = v(z)
        num = quad(lambda s: (v0 + k * s), 0.0, zz, epsabs=0, epsrel=1e-13)[0]  # int v^2 dt = int v dz
        assert math.sqrt(t0sq[i]) == pytest.approx(t0, rel=1e-12)
        assert 1.0 / s2[i] == pytest.approx(num / t0, rel=1e-12)
    t0sq, s2 = survey.traveltime_tables(np.array([400.0]), ("const", 2000.0))
    assert t0sq[0] == pytest.approx(0.04, rel=1e-15) and s2[0] == pytest.approx(2.5e-7, rel=1e-15)


def test_aperture_table_angle():
    z = np.array([10.0, 400.0, 2000.0])
    t0sq, s2 = survey.traveltime_tables(z, ("const", 2000.0))
    assert np.array_equal(survey.aperture_table(t0sq, s2, 45.0), (z * z).astype(np.float32))
    r2 = survey.aperture_table(t0sq, s2, 60.0)
    assert np.allclose(np.sqrt(r2.astype(np.float64)) / z, math.sqrt(3.0), rtol=1e-7)


def test_offset_bins_split_spread():
    p = survey.make_line2d(1)
    h = np.abs(p.src[:, 0].astype(np.float64) - p.rec[:, 0])
    assert np.all(np.diff(p.bin) >= 0)
    for b in range(8):
        hb = np.unique(h[p.bin == b])
        assert len(hb) == 3 and np.all((hb >= 75 * b) & (hb < 75 * (b + 1)))


def test_quantise_matches_torch_rounding():
    import torch

    rng = np.random.default_rng(0)
    d = (rng.standard_normal((5, 64)) * np.array([1, 1e-3, 1e3, 0, 7])[:, None]).astype(np.float32)
    for kind, tdt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
        bits, sig, deq = survey.quantise(d, kind)
        assert sig[3] == 1.0
        ref = torch.from_numpy(d / sig[:, None]).to(tdt)
        assert np.array_equal(bits, ref.view(torch.int16).numpy().view(np.uint16))
        assert np.allclose(deq, ref.to(torch.float64).numpy() * sig[:, None].astype(np.float64), rtol=0, atol=0)
